"""GPU parity of the post-integrator imaging (ddx_image_*, Sec. 3.3, 3.4, App. A.1)
against the FP64 oracle (oracle/imaging.py): ragged direction tiles and window
tiles, a row step with a window offset, F from 0 to 8, spans wider than the
32-window LDS tile allows (the 4-window kernel), bins beyond kmax, P-only and
E-only calls, and end to end from plane-wave chirp voltages through the GPU
pre-integrator: the on-bin sum N M (M - 1) / 2 (Eq. pthsum) and the peak of E at
the source (Eq. eth).
Bound: FP32 weights, bins and sums over pairs x taps terms -> the error of P is
held to 1e-5 of sqrt(pairs x taps) x the RMS of the bins."""
import numpy as np
import pytest
import torch

from gpu_helpers import say
from oracle import imaging as oim
from paper_1109_3186_amd import Chirp, Image
import synth

pytestmark = pytest.mark.gpu

TOL = 1e-5
C = 299792458.0


def _layout(rng, M, radius, height):
    r = radius * np.sqrt(rng.uniform(0, 1, M))
    ph = rng.uniform(0, 2 * np.pi, M)
    return np.stack([r * np.cos(ph), r * np.sin(ph), rng.uniform(-height, height, M)], axis=1)


def _check(S, ant, pix, fdot, f_s, N, L, kmax, F, first, w_step, want=(True, True)):
    dev = torch.device("cuda:0")
    x = torch.from_numpy(np.ascontiguousarray(S.astype(np.complex64))).to(dev)
    with Image(ant, pix, fdot, f_s, N, L, kmax, F) as h:
        p, e = h.run(x, first_window=first, w_step=w_step, want_p=want[0], want_e=want[1])
        torch.cuda.synchronize()
    ref = oim.image(S[::w_step], ant, pix, fdot, f_s, N, L, kmax, F, first_window=first, w_step=w_step)
    scale = np.sqrt(S.shape[1] * (2 * F + 1) * np.mean(np.abs(S) ** 2))
    tol = TOL * scale
    if p is not None:
        got = p.cpu().numpy()
        assert got.shape == ref.shape
        err = np.max(np.abs(got - ref))
        say("P: max error %.3e (bound %.3e), max |P| %.3e" % (err, tol, np.max(np.abs(ref))))
        assert err <= tol
    if e is not None:
        got_e = e.cpu().numpy()
        ref_e = np.abs(ref) ** 2
        assert got_e.shape == ref_e.shape
        err_e = np.max(np.abs(got_e - ref_e))
        bound = 2 * np.max(np.abs(ref)) * tol + tol * tol
        say("E: max error %.3e (bound %.3e)" % (err_e, bound))
        assert err_e <= bound
    return ref


@pytest.mark.parametrize("M,kmax,F,n_rows,first,w_step,n_pix", [
    (6, 20, 2, 70, 5, 3, 600),     # ragged direction tile, partial window tile
    (9, 12, 0, 40, 0, 1, 300),     # F = 0 (Eq. pth), two window tiles
    (4, 30, 8, 5, 1000, 2, 1),     # F = 8, one direction, window offset
    (7, 6, 3, 33, 17, 4, 257),     # taps beyond kmax at the band edge
])
def test_image_matches_oracle(gpu, M, kmax, F, n_rows, first, w_step, n_pix):
    rng = np.random.Generator(np.random.PCG64(7000 + M))
    N, L, f_s = 256, 16, 1e6
    ant = _layout(rng, M, 900.0, 25.0)
    pix = rng.uniform(-0.04, 0.04, (n_pix, 2))
    b_max = max(np.linalg.norm(ant[p] - ant[q]) for p in range(M) for q in range(p + 1, M))
    fdot = 0.8 * kmax * f_s * C / (N * b_max * 0.057)   # the band edge near the field edge
    nbl = M * (M - 1) // 2
    S = synth.noise_complex(rng, (n_rows, nbl, 2 * kmax + 1))
    say("image: M %d kmax %d F %d rows %d first %d step %d pix %d" % (M, kmax, F, n_rows, first, w_step, n_pix))
    _check(S, ant, pix, fdot, f_s, N, L, kmax, F, first, w_step)


def test_wide_spans_use_the_narrow_window_tile(gpu):
    """A tile whose directions spread a pair's tone over more than 256 bins needs
    more LDS per window than 32 windows allow; the 4-window kernel takes it."""
    rng = np.random.Generator(np.random.PCG64(7100))
    M, kmax, F, N, L, f_s = 3, 400, 1, 2048, 64, 1e6
    ant = np.array([[0.0, 0.0, 0.0], [1000.0, 0.0, 0.0], [0.0, 700.0, 5.0]])
    pix = np.stack([np.linspace(-0.1, 0.1, 300), np.zeros(300)], axis=1)
    fdot = 380 * f_s * C / (N * 1000.0 * 0.1)
    S = synth.noise_complex(rng, (9, 3, 2 * kmax + 1))
    say("image: wide spans, kmax %d" % kmax)
    _check(S, ant, pix, fdot, f_s, N, L, kmax, F, 2, 1)


@pytest.mark.parametrize("want", [(True, False), (False, True)])
def test_p_only_and_e_only(gpu, want):
    rng = np.random.Generator(np.random.PCG64(7200))
    M, kmax = 5, 10
    ant = _layout(rng, M, 500.0, 10.0)
    pix = rng.uniform(-0.03, 0.03, (40, 2))
    S = synth.noise_complex(rng, (6, 10, 2 * kmax + 1))
    _check(S, ant, pix, 5e10, 1e6, 128, 8, kmax, 2, 3, 1, want)


def test_end_to_end_on_bin_chirp(gpu):
    """Plane-wave chirp on a line of antennas with one bin per antenna step at the
    source: the GPU pre-integrator and image give N M (M - 1) / 2 at the source
    for F = 0 and F = 2, and E peaks there along l."""
    N, L, f_s, spacing, l0 = 256, 16, 1e6, 300.0, 0.25
    fdot = f_s * C / (N * spacing * l0)
    M, kmax, w0 = 8, 9, 3
    pos = np.stack([np.arange(M) * spacing, np.zeros(M), np.zeros(M)], axis=1)
    t = (np.arange(N + 8 * L) - w0 * L) / f_s
    arrive = -pos[:, 0] * l0 / C
    s = np.exp(1j * np.pi * fdot * (t[None, :] - arrive[:, None]) ** 2)
    dev = torch.device("cuda:0")
    with Chirp(M, N, L, kmax, max_samples=s.shape[1]) as c:
        S = c.preintegrate(torch.from_numpy(s.astype(np.complex64)).to(dev))
    # the line resolves l only; the source is the middle direction
    grid = np.array([(l0 + dl, 0.0) for dl in (-0.02, -0.01, 0.0, 0.01, 0.02)])
    for F in (0, 2):
        with Image(pos, grid, fdot, f_s, N, L, kmax, F) as h:
            p, e = h.run(S[w0:w0 + 1], first_window=w0)
            torch.cuda.synchronize()
        p, e = p.cpu().numpy(), e.cpu().numpy()
        ideal = N * M * (M - 1) / 2
        say("F %d: P at the source %.6e + %.2e i (ideal %.0f)" % (F, p[0, 2].real, p[0, 2].imag, ideal))
        assert abs(p[0, 2] - ideal) <= 1e-5 * ideal
        assert int(np.argmax(e[0])) == 2


def test_bank_and_image_end_to_end(gpu):
    """The Chirpolator on the device end to end: plane-wave chirp voltages through
    the GPU bank of window lengths (with its factorisation) and the GPU image of
    each length with its own chirp rate; the fraction of the ideal coherent sum
    peaks at the true length and direction, and every length's image matches the
    oracle's bank + image on the same voltages."""
    import test_oracle_imaging as toi
    from oracle import chirpolator as och
    from paper_1109_3186_amd import ChirpBank
    s, pos, grid, f_s, n0, n_len, d_true, L, kmax, w0 = toi._bank_scene(41)
    x = torch.from_numpy(np.ascontiguousarray(s.astype(np.complex64))).to("cuda:0")
    with ChirpBank(6, n0, n_len, L, kmax, max_samples=s.shape[1]) as b:
        outs = b.run(x)
        ref_bank = och.bank_direct(s, n0, n_len, L, kmax)
        best = []
        for d, (S, R) in enumerate(zip(outs, ref_bank), start=1):
            fdot = f_s * f_s / (n0 * d)
            with Image(pos, np.array(grid), fdot, f_s, n0 * d, L, kmax, 2) as h:
                p, _ = h.run(S[w0:w0 + 1].contiguous(), first_window=w0, want_e=False)
                torch.cuda.synchronize()
            p = p.cpu().numpy()
            ref = oim.image(R[w0:w0 + 1], pos, grid, fdot, f_s, n0 * d, L, kmax, 2, first_window=w0)
            scale = n0 * d * 15
            err = np.max(np.abs(p - ref)) / scale
            say("length %d: max |P - oracle| / (N pairs) %.2e, best fraction %.3f" % (
                d, err, np.abs(p).max() / scale))
            assert err <= 1e-5
            frac = np.abs(p[0]) / scale
            best.append((frac.max(), d, int(np.argmax(frac))))
    top = max(best)
    assert top[1] == d_true and top[2] == 4 and top[0] > 0.7
