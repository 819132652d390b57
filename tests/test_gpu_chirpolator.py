"""GPU parity of the Chirpolator pre-integrator (ddx_chirp_*, Sec. 3.2 and App. A.3)
against the FP64 oracle (oracle/chirpolator.py): ragged pair and bin tiles, block
lengths that are not a multiple of the LDS chunk, a partial last block, L = 1 with a
single bin, the DFT of a mixed linear chirp against its closed form (Eq. phidn), and
the bank of window lengths n0 d with the factorisation (ddx_chirp_bank_*) against
every length computed from its definition.
Bound: FP32 products and block sums, FP64 moving sum -> 1e-5 of the output's RMS."""
import numpy as np
import pytest
import torch

from gpu_helpers import say
from oracle import chirpolator as och
from paper_1109_3186_amd import Chirp, ChirpBank
import synth

pytestmark = pytest.mark.gpu

TOL = 1e-5


def _run(s, n_win, L, kmax):
    dev = torch.device("cuda:0")
    x = torch.from_numpy(np.ascontiguousarray(s.astype(np.complex64))).to(dev)
    with Chirp(s.shape[0], n_win, L, kmax, max_samples=s.shape[1]) as c:
        out = c.preintegrate(x)
        torch.cuda.synchronize()
        return out.cpu().numpy()


@pytest.mark.parametrize("m_ant,n_win,L,kmax,extra", [(5, 160, 40, 37, 17), (20, 192, 32, 70, 0), (3, 24, 8, 0, 5),
                                                      (4, 6, 1, 0, 0), (12, 4000, 1000, 12, 999)])
def test_preintegrator_matches_oracle(gpu, m_ant, n_win, L, kmax, extra):
    nb = n_win // L + 6
    s = synth.noise_complex(np.random.Generator(np.random.PCG64(90 + m_ant)), (m_ant, nb * L + extra))
    say("chirpolator: M %d N %d L %d kmax %d, %d samples" % (m_ant, n_win, L, kmax, s.shape[1]))
    got = _run(s, n_win, L, kmax)
    ref = och.preintegrate(s, n_win, L, kmax)
    assert got.shape == ref.shape
    err = np.max(np.abs(got - ref)) / np.sqrt(np.mean(np.abs(ref) ** 2))
    say("max error / rms %.3e" % err)
    assert err <= TOL


def test_cic_across_segments(gpu):
    """More blocks than one CIC segment (256): windows that straddle segment starts
    must equal the oracle's single recursion."""
    s = synth.noise_complex(np.random.Generator(np.random.PCG64(97)), (3, 700 * 4 + 3))
    got = _run(s, 64, 4, 3)
    ref = och.preintegrate(s, 64, 4, 3)
    err = np.max(np.abs(got - ref)) / np.sqrt(np.mean(np.abs(ref) ** 2))
    say("CIC over 700 blocks: max error / rms %.3e" % err)
    assert got.shape == ref.shape and err <= TOL


def test_mixed_chirp_closed_form_on_gpu(gpu):
    """Two antennas receive a linear chirp, q later by tau: the first complete
    window's bins are Phi(k - k0) D_N(k - k0), k0 = fdot tau N / f_s (Eq. phidn)."""
    f_s, n_win, L, tau, k0 = 1e6, 4096, 256, 2.5e-6, 3.37
    fdot = k0 * f_s / (tau * n_win)
    s = np.stack([och.linear_chirp(n_win, fdot, f_s), och.linear_chirp(n_win, fdot, f_s, tau)])
    got = _run(s, n_win, L, 12)[0, 0]
    ref = och.mixed_chirp_dft(och.bins(12), n_win, fdot, tau, f_s)
    err = np.max(np.abs(got - ref)) / n_win
    say("mixed chirp: peak |S| / N %.4f, max error / N %.2e" % (np.max(np.abs(got)) / n_win, err))
    assert err <= 2e-6


def test_short_stream_and_bad_arguments(gpu):
    from paper_1109_3186_amd import DdxError
    with Chirp(3, 64, 16, 4, max_samples=1000) as c:
        assert c.output_shape(63) == (0, 3, 9)
        x = torch.zeros((3, 63), dtype=torch.complex64, device="cuda:0")
        assert c.preintegrate(x).shape == (0, 3, 9)
        with pytest.raises(DdxError):
            c.preintegrate(torch.zeros((3, 1001), dtype=torch.complex64, device="cuda:0"))
        with pytest.raises(DdxError):
            c.preintegrate(torch.zeros((2, 100), dtype=torch.complex64, device="cuda:0"))


@pytest.mark.parametrize("m_ant,n0,n_len,L,kmax", [(4, 24, 6, 8, 5), (10, 64, 8, 16, 20), (3, 8, 12, 8, 3)])
def test_bank_matches_oracle(gpu, m_ant, n0, n_len, L, kmax):
    nb = n0 * n_len // L + 7
    s = synth.noise_complex(np.random.Generator(np.random.PCG64(98 + m_ant)), (m_ant, nb * L + 3))
    say("chirpolator bank: M %d n0 %d lengths %d L %d kmax %d" % (m_ant, n0, n_len, L, kmax))
    dev = torch.device("cuda:0")
    x = torch.from_numpy(np.ascontiguousarray(s.astype(np.complex64))).to(dev)
    with ChirpBank(m_ant, n0, n_len, L, kmax, max_samples=s.shape[1]) as b:
        outs = b.run(x)
        torch.cuda.synchronize()
        got = [o.cpu().numpy() for o in outs]
    ref = och.bank_direct(s, n0, n_len, L, kmax)
    for d, (g, r) in enumerate(zip(got, ref), start=1):
        assert g.shape == r.shape, d
        err = np.max(np.abs(g - r)) / np.sqrt(np.mean(np.abs(r) ** 2))
        assert err <= TOL, (d, err)
    say("bank: all %d lengths within %.0e" % (n_len, TOL))


def _run_budget(s, n_win, L, kmax, budgets):
    dev = torch.device("cuda:0")
    x = torch.from_numpy(np.ascontiguousarray(s.astype(np.complex64))).to(dev)
    with Chirp(s.shape[0], n_win, L, kmax, max_samples=s.shape[1]) as c:
        c.set_pair_bins(budgets)
        out = c.preintegrate(x)
        torch.cuda.synchronize()
        return out.cpu().numpy()


@pytest.mark.parametrize("kind", ["geometry", "two_groups"])
def test_pair_bin_budgets(gpu, kind):
    """Per-pair bin budgets: bins beyond a pair's budget are exactly zero, the others
    equal the oracle; 'two_groups' makes whole (pair tile, bin tile) blocks skip."""
    m_ant, n_win, L, kmax = 20, 192, 32, 70
    rng = np.random.Generator(np.random.PCG64(120))
    s = synth.noise_complex(rng, (m_ant, (n_win // L + 6) * L + 11))
    nbl = m_ant * (m_ant - 1) // 2
    if kind == "geometry":
        budgets = och.pair_bin_budgets(synth.antenna_positions(rng, m_ant, 3000.0), kmax)
    else:
        budgets = np.full(nbl, 5, dtype=np.int32)
        budgets[rng.permutation(nbl)[:64]] = kmax
    got = _run_budget(s, n_win, L, kmax, budgets)
    ref = och.preintegrate(s, n_win, L, kmax, pair_kmax=budgets)
    ks = och.bins(kmax)
    beyond = np.abs(ks)[None, :] > budgets[:, None]
    assert np.all(got[:, beyond] == 0)
    err = np.max(np.abs(got - ref)) / np.sqrt(np.mean(np.abs(ref[:, ~beyond]) ** 2))
    say("budgets (%s): %d of %d pair-bins computed, max error / rms %.3e" % (kind, (~beyond).sum(), beyond.size, err))
    assert err <= TOL


@pytest.mark.parametrize("kind", ["random", "zero"])
def test_bank_with_pair_bin_budgets(gpu, kind):
    """Budgets on a bank; 'zero' keeps only bin 0, so the lengths d > 1 (whose bin 0
    is factorised) launch no partial-DFT tile at all.  Clearing the budgets again
    restores the full output."""
    m_ant, n0, n_len, L, kmax = 10, 64, 8, 16, 20
    rng = np.random.Generator(np.random.PCG64(121))
    s = synth.noise_complex(rng, (m_ant, (n0 * n_len // L + 5) * L))
    nbl = m_ant * (m_ant - 1) // 2
    if kind == "random":
        budgets = rng.integers(0, kmax + 1, nbl).astype(np.int32)
    else:
        budgets = np.zeros(nbl, dtype=np.int32)
    x = torch.from_numpy(np.ascontiguousarray(s.astype(np.complex64))).to("cuda:0")
    with ChirpBank(m_ant, n0, n_len, L, kmax, max_samples=s.shape[1]) as b:
        b.set_pair_bins(budgets)
        got = [o.cpu().numpy() for o in b.run(x)]
        b.set_pair_bins(None)
        full = [o.cpu().numpy() for o in b.run(x)]
    for d, (g, f) in enumerate(zip(got, full), start=1):
        ref = och.preintegrate(s, n0 * d, L, kmax, pair_kmax=budgets)
        err = np.max(np.abs(g - ref)) / np.sqrt(np.mean(np.abs(ref) ** 2))
        assert err <= TOL, (d, err)
        ref = och.preintegrate(s, n0 * d, L, kmax)
        err = np.max(np.abs(f - ref)) / np.sqrt(np.mean(np.abs(ref) ** 2))
        assert err <= TOL, (d, "cleared", err)


def test_pair_bin_budget_rejected(gpu):
    from paper_1109_3186_amd import DdxError
    with Chirp(3, 64, 16, 4, max_samples=1000) as c:
        with pytest.raises(DdxError):
            c.set_pair_bins(np.array([4, 5, 1], dtype=np.int32))
        c.set_pair_bins(None)


def test_many_antennas_per_pair_tile(gpu):
    """100 antennas: a tile of 64 pairs reads up to 65 antennas in row-major order and
    up to 128 once random budgets reorder the pairs (the staged-antenna limit)."""
    m_ant, n_win, L, kmax = 100, 64, 16, 3
    rng = np.random.Generator(np.random.PCG64(130))
    s = synth.noise_complex(rng, (m_ant, (n_win // L + 3) * L))
    x = torch.from_numpy(np.ascontiguousarray(s.astype(np.complex64))).to("cuda:0")
    budgets = rng.integers(0, kmax + 1, m_ant * (m_ant - 1) // 2).astype(np.int32)
    with Chirp(m_ant, n_win, L, kmax, max_samples=s.shape[1]) as c:
        full = c.preintegrate(x).cpu().numpy()
        c.set_pair_bins(budgets)
        part = c.preintegrate(x).cpu().numpy()
    for got, bud in ((full, None), (part, budgets)):
        ref = och.preintegrate(s, n_win, L, kmax, pair_kmax=bud)
        err = np.max(np.abs(got - ref)) / np.sqrt(np.mean(np.abs(ref) ** 2))
        say("100 antennas (%s): max error / rms %.3e" % ("budgets" if bud is not None else "full", err))
        assert err <= TOL
