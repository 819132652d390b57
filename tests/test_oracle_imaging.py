"""Pins of the post-integrator imaging oracle (oracle/imaging.py).

The bins are not made by the imaging code: the tests synthesise the voltages of a
linear chirp arriving as a plane wave from a chosen direction (each antenna's
arrival time from its position, written here), run the pinned pre-integrator
oracle, and check the image against what Sec. 3.3 and 3.4 fix:

* with every pair's tone on a bin (integer k0), P at the true direction is
  N M (M - 1) / 2 (Eq. pthsum), for F = 0 and for wider filters (D_N vanishes at
  the other integers);
* bins beyond kmax drop out pair by pair;
* with off-bin tones the matched filter returns sum D_N(x)^2 / N per pair, real;
* E = |P|^2 peaks at the true direction of a grid (Eq. eth), in 1-D and 3-D arrays.
"""
import numpy as np
import pytest

from oracle import chirpolator as ch
from oracle import imaging as im

C = 299792458.0


def _plane_wave_chirp(pos, n_samp, fdot, f_s, l, m, origin):
    """s_p[n] = exp(pi i fdot (t - a_p)^2), t = (n - origin) / f_s, where a_p is when
    the wavefront from (l, m) passes antenna p, relative to the array origin, after
    the delay of the pointing direction (0, 0, 1) is taken out."""
    pos = np.asarray(pos, dtype=np.float64)
    d = np.array([l, m, np.sqrt(1.0 - l * l - m * m)])
    arrive = -(pos @ d) / C + pos[:, 2] / C
    t = (np.arange(n_samp) - origin) / f_s
    return np.exp(1j * np.pi * fdot * (t[None, :] - arrive[:, None]) ** 2), arrive


def _line_array(M, spacing):
    return np.stack([np.arange(M) * spacing, np.zeros(M), np.zeros(M)], axis=1)


# a 1-D array whose pair tones sit on bins: fdot N spacing l0 / (f_s c) = 1 bin per
# antenna step at the direction l0
N, L, F_S = 128, 16, 1.0e6
SPACING, L0 = 300.0, 0.25
FDOT = F_S * C / (N * SPACING * L0)


def _bins_of_line(M, kmax, origin_window, n_windows=3):
    pos = _line_array(M, SPACING)
    n_samp = N + (origin_window + n_windows) * L
    s, _ = _plane_wave_chirp(pos, n_samp, FDOT, F_S, L0, 0.0, origin_window * L)
    S = ch.preintegrate(s, N, L, kmax)
    return pos, S


@pytest.mark.parametrize("F", [0, 2])
def test_on_bin_tones_sum_to_n_pairs(F):
    """Eq. pthsum: every pair contributes D_N(0) = N at the true direction."""
    M, w0 = 6, 2
    pos, S = _bins_of_line(M, kmax=M, origin_window=w0)
    P = im.image(S[w0:w0 + 1], pos, [(L0, 0.0)], FDOT, F_S, N, L, M, F, first_window=w0)
    assert abs(P[0, 0] - N * M * (M - 1) / 2) < 1e-8 * N * M * M


def test_bins_beyond_kmax_drop_out():
    """Pair (p, q) sits at k0 = p - q bins; with kmax = 2 only |p - q| <= 2 remain."""
    M, w0, kmax = 6, 1, 2
    pos, S = _bins_of_line(M, kmax=kmax, origin_window=w0)
    P = im.image(S[w0:w0 + 1], pos, [(L0, 0.0)], FDOT, F_S, N, L, kmax, 1, first_window=w0)
    kept = sum(1 for p in range(M) for q in range(p + 1, M) if q - p <= kmax)
    assert abs(P[0, 0] - N * kept) < 1e-8 * N * M * M


def test_window_reference_matters():
    """The same chirp imaged in a window that does not start at the chirp's origin
    loses coherence (the window phase and the linear term no longer match)."""
    M, w0 = 6, 2
    pos, S = _bins_of_line(M, kmax=M, origin_window=w0)
    P = im.image(S[w0 - 1:w0], pos, [(L0, 0.0)], FDOT, F_S, N, L, M, 0, first_window=w0 - 1)
    assert abs(P[0, 0]) < 0.9 * N * M * (M - 1) / 2


def _random_3d(rng, M, radius, height):
    r = radius * np.sqrt(rng.uniform(0, 1, M))
    ph = rng.uniform(0, 2 * np.pi, M)
    return np.stack([r * np.cos(ph), r * np.sin(ph), rng.uniform(-height, height, M)], axis=1)


def test_off_bin_matched_filter_3d():
    """Sec. 3.4 with off-bin tones in a 3-D array: at the true direction each pair
    returns sum_t D_N(k0' + t - k0)^2 / N (X = Phi D_N, weight = conj(Phi) D_N / N),
    a real sum; the offsets are computed here from the antennas' arrival times."""
    rng = np.random.Generator(np.random.PCG64(3186))
    M, F, kmax, w0 = 5, 3, 40, 1
    pos = _random_3d(rng, M, 1500.0, 40.0)
    l0, m0 = 0.07, -0.05
    fdot = 3.0e10
    s, arrive = _plane_wave_chirp(pos, N + 4 * L, fdot, F_S, l0, m0, w0 * L)
    S = ch.preintegrate(s, N, L, kmax)
    P = im.image(S[w0:w0 + 1], pos, [(l0, m0)], fdot, F_S, N, L, kmax, F, first_window=w0)
    expect = 0.0
    for p in range(M):
        for q in range(p + 1, M):
            k0 = fdot * (arrive[q] - arrive[p]) * N / F_S
            assert abs(k0) + F < kmax
            x = np.rint(k0) + np.arange(-F, F + 1) - k0
            expect += np.sum((np.sin(np.pi * x) / np.sin(np.pi * x / N)) ** 2) / N
    assert abs(P[0, 0] - expect) < 1e-9 * expect


@pytest.mark.parametrize("three_d", [False, True])
def test_energy_peaks_at_true_direction(three_d):
    """Eq. eth: E over a grid of directions is largest at the source."""
    rng = np.random.Generator(np.random.PCG64(11 + three_d))
    M, kmax, w0 = 6, 24, 1
    pos = _random_3d(rng, M, 1200.0, 30.0 if three_d else 0.0)
    l0, m0 = 0.04, 0.02
    fdot = 2.0e10
    s, _ = _plane_wave_chirp(pos, N + 3 * L, fdot, F_S, l0, m0, w0 * L)
    S = ch.preintegrate(s, N, L, kmax)
    grid = [(l0 + dl, m0 + dm) for dl in (-0.02, 0.0, 0.02) for dm in (-0.02, 0.0, 0.02)]
    E = im.energy(im.image(S[w0:w0 + 1], pos, grid, fdot, F_S, N, L, kmax, 2, first_window=w0))
    assert int(np.argmax(E[0])) == 4


def test_rows_follow_window_index():
    """A w_step > 1 selection of rows gives the same images as imaging the rows one
    at a time with their own window index."""
    rng = np.random.Generator(np.random.PCG64(5))
    M, kmax = 4, 6
    pos = _random_3d(rng, M, 800.0, 10.0)
    S = rng.normal(size=(7, M * (M - 1) // 2, 2 * kmax + 1)) + 1j * rng.normal(size=(7, M * (M - 1) // 2, 2 * kmax + 1))
    pix = [(0.01, -0.02), (-0.03, 0.0)]
    P = im.image(S[::3], pos, pix, 1e10, F_S, N, L, kmax, 1, first_window=5, w_step=3)
    for i in range(3):
        Pi = im.image(S[3 * i:3 * i + 1], pos, pix, 1e10, F_S, N, L, kmax, 1, first_window=5 + 3 * i)
        np.testing.assert_allclose(P[i], Pi[0], rtol=1e-13)


def _bank_scene(seed):
    """Six antennas within 1.5 km, a chirp of rate f_s^2 / N_true (it sweeps the
    whole band in one window of N_true samples, Sec. 3.2) from (l0, m0) whose
    quadratic origin is at the start of window w0."""
    rng = np.random.Generator(np.random.PCG64(seed))
    f_s, n0, n_len, d_true, L, kmax, w0 = 8e6, 64, 4, 3, 16, 12, 2
    pos = _random_3d(rng, 6, 1500.0, 10.0)
    l0, m0 = 0.06, -0.04
    fdot = f_s * f_s / (n0 * d_true)
    n_samp = n0 * n_len + (w0 + 2) * L
    s, _ = _plane_wave_chirp(pos, n_samp, fdot, f_s, l0, m0, w0 * L)
    grid = [(l0 + dl, m0 + dm) for dl in (-0.02, 0.0, 0.02) for dm in (-0.02, 0.0, 0.02)]
    return s, pos, grid, f_s, n0, n_len, d_true, L, kmax, w0


def test_bank_and_image_find_the_chirp_rate_and_direction():
    """The Chirpolator end to end on the CPU: the bank of window lengths n0 d (one per
    chirp rate, fdot_d = f_s^2 / (n0 d)) and the image of each length's window w0
    with its own rate.  Each length's |P| is compared as a fraction of its ideal
    coherent sum N_d M (M - 1) / 2 (Eq. pthsum), which grows with N_d: the largest
    fraction is at the true length and the true direction, and is near 1 there."""
    s, pos, grid, f_s, n0, n_len, d_true, L, kmax, w0 = _bank_scene(41)
    bank = ch.bank_direct(s, n0, n_len, L, kmax)
    npairs = 15
    best = []
    for d, S in enumerate(bank, start=1):
        P = im.image(S[w0:w0 + 1], pos, grid, f_s * f_s / (n0 * d), f_s, n0 * d, L, kmax, 2, first_window=w0)
        frac = np.abs(P[0]) / (n0 * d * npairs)
        best.append((frac.max(), d, int(np.argmax(frac))))
    top = max(best)
    assert top[1] == d_true and top[2] == 4 and top[0] > 0.7
