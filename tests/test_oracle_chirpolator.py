"""Pins of the Chirpolator pre-integrator oracle (oracle/chirpolator.py): the
block-CIC recursion against the sliding-DFT definition, the DFT of a mixed
linear chirp against its closed form (Eqs. phidn, dn, phipq1), the k = 0 bin
against the integrate-and-dump of the correlator oracle, the factorisation
identity and the op-count claims of App. A.3 against the paper's numbers."""
import math
import os

import numpy as np
import pytest

from oracle import chirpolator as ch
from oracle import correlate_dumps
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden(name):
    with open(os.path.join(GOLDEN, "paper_constants.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            k, v, tol, _cite = line.split()
            if k == name:
                return float(v), float(tol)
    raise KeyError(name)


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


@pytest.mark.parametrize("n_win,L,kmax", [(60, 12, 3), (48, 48, 5), (64, 8, 7)])
def test_block_cic_is_the_sliding_dft(n_win, L, kmax):
    """Eq. block_cic from zero state equals, block by block, the DFT of the last N
    samples (brute force over the window), including the ramp-up blocks."""
    x = synth.noise_complex(_rng(1), (10 * L,))
    ks = ch.bins(kmax)
    s = ch.block_cic(ch.block_partial_dft(x, n_win, L, ks), n_win, L)
    ref = ch.sliding_dft(x, n_win, L, ks)
    np.testing.assert_allclose(s, ref, atol=1e-11)
    # and the full windows against an O(N^2) DFT of the window with phase from sample 0
    for m in range(n_win // L - 1, 10):
        lo = (m + 1) * L - n_win
        for j, k in enumerate(ks):
            direct = sum(x[n] * np.exp(-2j * np.pi * n * k / n_win) for n in range(lo, lo + n_win))
            assert abs(s[m, j] - direct) < 1e-10


@pytest.mark.parametrize("k0", [3.37, -5.81, 4.0])
def test_mixed_chirp_matches_closed_form(k0):
    """Sec. 3.2: mixing a linear chirp with its copy delayed by tau gives a tone at
    k0 = fdot tau N / f_s, and its N-point DFT is Phi(k - k0) D_N(k - k0) (Eqs. phidn,
    dn, phipq1).  An integer k0 puts D_N(0) = N in one bin and zeros elsewhere."""
    f_s, n_win, tau = 1e6, 4096, 2.5e-6
    fdot = k0 * f_s / (tau * n_win)
    sp = ch.linear_chirp(n_win, fdot, f_s)
    sq = ch.linear_chirp(n_win, fdot, f_s, tau)   # antenna q receives it tau later
    x = ch.mix(np.stack([sp, sq]), 0, 1)
    ks = ch.bins(12)
    got = ch.block_cic(ch.block_partial_dft(x, n_win, n_win, ks), n_win, n_win)[0]
    ref = ch.mixed_chirp_dft(ks, n_win, fdot, tau, f_s)
    np.testing.assert_allclose(got, ref, atol=1e-7 * n_win)
    if float(k0).is_integer():
        ratio, tol = _golden("dirichlet_at_zero_over_N")
        j = int(np.where(ks == int(k0))[0][0])
        assert abs(abs(got[j]) / n_win - ratio) <= tol + 1e-12
        assert np.max(np.abs(np.delete(got, j))) < 1e-7 * n_win


def test_dirichlet_kernel_is_the_geometric_sum():
    n = 37
    for x in [0.0, 0.3, 1.0, -2.5, 7.0]:
        direct = sum(np.exp(-2j * np.pi * t * x / n) for t in range(n))
        closed = np.exp(-1j * np.pi * x * (n - 1) / n) * ch.dirichlet(np.array([x]), n)[0]
        assert abs(direct - closed) < 1e-11


def test_k0_bin_of_a_block_is_the_integrate_and_dump():
    """At k = 0 the block partial DFT of x_pq is the correlator's dump V_pq[m]."""
    m_ant, L, n_win = 4, 25, 100
    s = synth.noise_complex(_rng(2), (m_ant, 8 * L))
    dumps = correlate_dumps(s, L)
    for p, q in ch.pairs(m_ant):
        v = ch.block_partial_dft(ch.mix(s, p, q), n_win, L, [0])[:, 0]
        np.testing.assert_allclose(v, dumps[:, p, q], atol=1e-12)


@pytest.mark.parametrize("n0,d,k,D", [(8, 2, 2, 2), (8, 4, 6, 2), (5, 6, 9, 3), (6, 4, 8, 4)])
def test_factorisation_identity(n0, d, k, D):
    """Bin k of the length-N0 d DFT equals the sum of D adjacent bins k/D of length
    N0 d/D.  The printed shift d' N0 is right when d = D (the paper's example)."""
    x = synth.noise_complex(_rng(3), (200,))
    end = 150
    full = ch.window_dft(x, end, n0 * d, k)
    assert abs(ch.factorised_bin(x, end, n0, d, k, D) - full) < 1e-11
    printed = sum(ch.window_dft(x, end - j * n0, n0 * d // D, k // D) for j in range(D))
    assert (abs(printed - full) < 1e-11) == (d == D)


def test_factorisable_fraction_matches_the_paper():
    want, tol = _golden("factorisable_fraction")
    frac = ch.factorisable_fraction(500, 500)
    assert abs(frac - (1 - 6 / math.pi ** 2)) < 0.005
    assert abs(frac - want) <= tol


def test_negative_bin_sharing():
    rng = _rng(4)
    for _ in range(20):
        a, b, c, d = rng.standard_normal(4)
        rk, rmk, mults, adds = ch.pos_neg_products(a, b, c, d)
        assert abs(rk - (a + 1j * b) * (c - 1j * d)) < 1e-14
        assert abs(rmk - (a + 1j * b) * (c + 1j * d)) < 1e-14
    want, tol = _golden("pos_neg_saving")
    assert abs((12 - (mults + adds)) / 12 - want) <= tol


def test_preintegrate_shape_and_pairs():
    m_ant, L, n_win, kmax = 4, 10, 40, 2
    s = synth.noise_complex(_rng(5), (m_ant, 12 * L))
    out = ch.preintegrate(s, n_win, L, kmax)
    assert out.shape == (12 - n_win // L + 1, m_ant * (m_ant - 1) // 2, 2 * kmax + 1)
    p, q = ch.pairs(m_ant)[4]
    ref = ch.sliding_dft(ch.mix(s, p, q), n_win, L, ch.bins(kmax))[n_win // L - 1:]
    np.testing.assert_allclose(out[:, 4], ref, atol=1e-11)


def test_bank_factorisation_at_block_resolution():
    """The bank built with App. A.3's factorisation (block-resolution window offsets)
    equals every length computed from its definition; at these sizes 23 of the
    6 x 11 (d, k) bins are factorised (d = 2: 5, 3: 3, 4: 5, 5: 3, 6: 7)."""
    m_ant, n0, n_len, L, kmax = 3, 12, 6, 4, 5
    s = synth.noise_complex(_rng(6), (m_ant, (n0 * n_len // L + 5) * L))
    direct = ch.bank_direct(s, n0, n_len, L, kmax)
    fact = ch.bank_factorised(s, n0, n_len, L, kmax)
    for a, b in zip(direct, fact):
        assert a.shape == b.shape
        np.testing.assert_allclose(b, a, atol=1e-10)
    n_fact = sum(1 for d in range(1, n_len + 1) for k in range(-kmax, kmax + 1) if math.gcd(abs(k), d) > 1)
    assert n_fact == 23


@pytest.mark.parametrize("c", [5, 6, 7, 8, 12, 13, 31, 64])
def test_gauss_sum_closed_forms(c):
    """G(1/c, c) is the quadratic Gauss sum: sqrt(c), 0, i sqrt(c) or (1 + i) sqrt(c)
    for c = 1, 2, 3, 0 mod 4; G(0, L) = L and |G(a, L)| < L otherwise (App. A.2)."""
    g = ch.gauss_sum(1.0 / c, c)
    expect = {1: np.sqrt(c), 2: 0.0, 3: 1j * np.sqrt(c), 0: (1 + 1j) * np.sqrt(c)}[c % 4]
    assert abs(g - expect) < 1e-9 * c
    assert abs(ch.gauss_sum(0.0, c) - c) < 1e-12
    assert ch.coherence_loss(0.3 / c ** 2, c) < 1.0


def test_coherence_loss_falls_with_the_block_length():
    """For a fixed chirp rate a, longer blocks lose more (eta decreasing in L), and
    eta is the magnitude of the k = 0 block partial DFT of the chirp over L."""
    a = 2e-6
    etas = [ch.coherence_loss(a, L) for L in (64, 256, 512, 1024)]
    assert all(x > y for x, y in zip(etas, etas[1:])) and etas[0] > 0.99
    L = 300
    x = np.exp(2j * np.pi * a * np.arange(L) ** 2)
    v = ch.block_partial_dft(x, L, L, [0])[0, 0]
    assert abs(abs(v) / L - ch.coherence_loss(a, L)) < 1e-12


def test_pair_bin_budgets_hand_example():
    """A 3-4-5 triangle: baselines 3, 4 and 5 (pairs (0,1), (0,2), (1,2)), k_max 10:
    budgets ceil(10 b / 5) = 6, 8, 10."""
    pos = np.array([[0.0, 0.0], [3.0, 0.0], [0.0, 4.0]])
    assert list(ch.pair_bin_budgets(pos, 10)) == [6, 8, 10]
