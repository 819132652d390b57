"""Pins of the Chimageator oracle (oracle/chimageator.py): gridding against the
per-pair definition, the spatial DFT against numpy's FFT of the zero-padded
spacings (a library routine), the phase term against the closed form of a spatial
tone's DFT, and the trajectory sum of a chirp arriving on a uniform linear array,
whose mixed products are synthesised here from the antennas' arrival times: the
true (end bin, duration, start) gives the largest |P| of a grid of trials and
nearly the ideal (M - 1) T_b."""
import numpy as np
import pytest

from oracle import chimageator as cg


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def test_grid_is_the_per_pair_definition():
    rng = _rng(1)
    s = rng.normal(size=(5, 40)) + 1j * rng.normal(size=(5, 40))
    G = cg.grid_blocks(s, 8)
    for m in range(5):
        for l in range(1, 5):
            ref = sum(s[p, n] * np.conj(s[p + l, n]) for p in range(5 - l) for n in range(8 * m, 8 * m + 8))
            assert abs(G[m, l - 1] - ref / ((5 - l) * 8)) < 1e-12
    Gu = cg.grid_blocks(s, 8, weights="uniform")
    assert np.allclose(Gu[:, 1] / 3, G[:, 1], atol=1e-14)


@pytest.mark.parametrize("M,n_s", [(4, 4), (9, 16), (16, 64)])
def test_spatial_dft_is_the_padded_fft(M, n_s):
    rng = _rng(M)
    G = rng.normal(size=(3, M - 1)) + 1j * rng.normal(size=(3, M - 1))
    pad = np.zeros((3, n_s), dtype=complex)
    pad[:, 1:M] = G
    assert np.allclose(cg.spatial_dft(G, n_s), np.fft.fft(pad, axis=1), atol=1e-12)


def test_phase_of_a_spatial_tone():
    """G_l = exp(2 pi i l x0 / N_s): Y_k = Phi(x0 - k) sin(pi (M - 1) (x0 - k) / N_s) /
    sin(pi (x0 - k) / N_s), the geometric sum written out."""
    M, n_s, x0 = 12, 32, 7.3
    G = np.exp(2j * np.pi * np.arange(1, M) * x0 / n_s)[None, :]
    Y = cg.spatial_dft(G, n_s)[0]
    for k in range(n_s):
        x = x0 - k
        ref = cg.phase(x, M, n_s) * np.sin(np.pi * (M - 1) * x / n_s) / np.sin(np.pi * x / n_s)
        assert abs(Y[k] - ref) < 1e-10


def ula_chirp(M, n_samp, f_s, t_samples, tau1, start):
    """Voltages of a chirp sweeping the band f_s in t_samples samples (fdot = f_s^2 /
    t_samples), starting at sample `start` and lasting t_samples samples, reaching
    antenna p a time p tau1 late (zero outside its duration at each antenna)."""
    fdot = f_s * f_s / t_samples
    t = (np.arange(n_samp) - start) / f_s
    tp = t[None, :] - (np.arange(M) * tau1)[:, None]
    on = (tp >= 0) & (tp < t_samples / f_s)
    return np.where(on, np.exp(1j * np.pi * fdot * tp ** 2), 0)


def test_trajectory_finds_the_chirp():
    M, n_s, L, f_s = 16, 32, 16, 1e6
    tb, m0 = 24, 5
    t_samples = tb * L
    k_end = 9.0
    tau1 = k_end / (n_s * f_s)       # k_end = N_s tau_1 f_s
    s = ula_chirp(M, (m0 + tb + 6) * L, f_s, t_samples, tau1, m0 * L)
    Y = cg.spatial_dft(cg.grid_blocks(s, L), n_s)
    best = cg.trajectory(Y, M, n_s, k_end, tb, m0, L)
    assert abs(best) > 0.85 * (M - 1) * tb
    for dk in (-1.0, 1.0):
        assert abs(cg.trajectory(Y, M, n_s, k_end + dk, tb, m0, L)) < abs(best)
    # another duration (chirp rate, i.e. DM) with the same end bin: another slope
    for dt in (-6, 6):
        assert abs(cg.trajectory(Y, M, n_s, k_end, tb + dt, m0, L)) < abs(best)
    for dm in (-2, 2):
        assert abs(cg.trajectory(Y, M, n_s, k_end, tb, m0 + dm, L)) < abs(best)
    P = cg.trajectories(Y, M, n_s, [(k_end, tb), (k_end + 2, tb)], L)
    assert int(np.argmax(np.abs(P[0]))) == m0 and np.all(P[:, Y.shape[0] - tb + 1:] == 0)
    # over a grid of end bins x durations and every start, the true trial wins
    trials = [(k_end + dk, tb + dt) for dk in (-1.0, 0.0, 1.0) for dt in (-6, 0, 6)]
    Pg = np.abs(cg.trajectories(Y, M, n_s, trials, L))
    i, m = np.unravel_index(np.argmax(Pg), Pg.shape)
    assert trials[i] == (k_end, tb) and m == m0


@pytest.mark.parametrize("k_end,tb", [(9.0, 24), (5.3, 40), (17.0, 11)])
def test_trajectory_of_exact_spatial_tones(k_end, tb):
    """Single-sample blocks (L = 1) of the mixed products of a chirp without the
    tau^2 term (s_p[n] = exp(-2 pi i fdot tau_1 p t_n), so that s_p s_{p+l}^* =
    exp(2 pi i fdot tau_1 l t_n) exactly): each sample's spatial DFT is Phi(x) times
    the real sum sin(pi (M - 1) x / N_s) / sin(pi x / N_s), so the trajectory sum
    is real, sum_n of that amplitude at x_n = N_s u_n - rint(N_s u_n), u_n = fdot
    tau_1 t_n cycles per spacing (computed here from the chirp's parameters)."""
    M, n_s, f_s, m0 = 12, 32, 1e6, 3
    fdot = f_s * f_s / tb                  # sweeps f_s in tb samples
    tau1 = k_end / (n_s * f_s)
    t = (np.arange(m0 + tb + 2) - m0) / f_s
    s = np.exp(-2j * np.pi * fdot * tau1 * np.outer(np.arange(M), t))
    Y = cg.spatial_dft(cg.grid_blocks(s, 1), n_s)   # natural weights: G_l = the tone
    P = cg.trajectory(Y, M, n_s, k_end, tb, m0, 1)
    expect = 0.0
    for n in range(m0, m0 + tb):
        u = fdot * tau1 * (n - m0) / f_s
        x = n_s * u - np.rint(n_s * u)
        expect += (M - 1) if x == 0 else np.sin(np.pi * (M - 1) * x / n_s) / np.sin(np.pi * x / n_s)
    assert abs(P - expect) < 1e-9 * (M - 1) * tb


def test_gradient_sums_are_the_trajectories_of_each_duration():
    """App. B: for a gradient g, the duration-T sum is the trajectory ending at bin
    k_end = g T after T blocks (the same line in (block, bin))."""
    rng = _rng(31)
    M, n_s, L, nb = 10, 32, 8, 40
    Y = rng.normal(size=(nb, n_s)) + 1j * rng.normal(size=(nb, n_s))
    grads, lengths = [0.37, -0.81, 1.93], [3, 10, 25]
    P = cg.gradient_sums(Y, M, n_s, grads, lengths, L)
    for i, g in enumerate(grads):
        for j, T in enumerate(lengths):
            for m0 in (0, 7, nb - T):
                ref = cg.trajectory(Y, M, n_s, g * T, T, m0, L)
                assert abs(P[i, j, m0] - ref) < 1e-10 * T
            assert np.all(P[i, j, nb - T + 1:] == 0)


def test_cell_gridding_reduces_to_the_uniform_line():
    """Antennas at integer multiples of the spacing: the cells are the spacings and
    the cell gridding is the uniform-line gridding with natural weights; jittered
    positions keep each pair in its cell."""
    rng = _rng(40)
    M, L = 7, 6
    s = rng.normal(size=(M, 5 * L)) + 1j * rng.normal(size=(M, 5 * L))
    cells = cg.nearest_cells(np.arange(M) * 25.0, 25.0)
    assert sorted(cells) == list(range(1, M)) and all(len(cells[l]) == M - l for l in cells)
    np.testing.assert_allclose(cg.grid_blocks_cells(s, L, cells, M - 1), cg.grid_blocks(s, L), atol=1e-13)
    jit = np.arange(M) * 25.0 + rng.uniform(-5, 5, M)
    assert cg.nearest_cells(jit, 25.0) == cells


def test_cell_gridding_of_a_sparse_line_finds_the_chirp():
    """A non-uniform line (some positions missing, some doubled spacings): the
    chirp's spatial tone is still a tone over the cells, and the trajectory at the
    true end bin, duration and start is the largest over a grid of trials."""
    M, n_s, L, f_s = 10, 64, 16, 1e6
    tb, m0, k_end = 20, 4, 11.0
    pos_idx = np.array([0, 1, 3, 4, 7, 8, 11, 15, 16, 20])          # in units of the spacing
    tau1 = k_end / (n_s * f_s)
    fdot = f_s * f_s / (tb * L)
    n = (m0 + tb + 6) * L
    t = (np.arange(n) - m0 * L) / f_s
    tp = t[None, :] - (pos_idx * tau1)[:, None]
    s = np.where((tp >= 0) & (tp < tb * L / f_s), np.exp(1j * np.pi * fdot * tp ** 2), 0)
    cells = cg.nearest_cells(pos_idx * 30.0, 30.0)
    Y = cg.spatial_dft(cg.grid_blocks_cells(s, L, cells, 20), n_s)
    trials = [(k_end + dk, tb + dt) for dk in (-1.0, 0.0, 1.0) for dt in (-5, 0, 5)]
    # the phase of the sum over cells 1 .. 20 is that of a 21-element line
    P = np.abs(cg.trajectories(Y, 21, n_s, trials, L))
    i, m = np.unravel_index(np.argmax(P), P.shape)
    assert trials[i] == (k_end, tb) and m == m0


# ---- App. B: spectral smearing (2F + 1 bins), sampling (kappa_t), planar gridding ----


def test_tone_amplitude_and_phase_are_the_spatial_response():
    """Y_k of a spatial tone at k0 = k + x is Phi(x) S(x), at fractional and integer k0."""
    for M, n_s, x0 in [(12, 32, 7.3), (9, 16, 5.0)]:
        G = np.exp(2j * np.pi * np.arange(1, M) * x0 / n_s)[None, :]
        Y = cg.spatial_dft(G, n_s)[0]
        x = x0 - np.arange(n_s)
        assert np.allclose(Y, cg.phase(x, M, n_s) * cg.tone_amplitude(x, M, n_s), atol=1e-10)


def test_widened_trajectory_reduces_to_eq_chimg_pth_and_sums_parseval():
    """F = 0 at an integer k0 (a source at broadside, k_end = 0) is Eq. chimg_pth; with
    all N_s bins (odd N_s, F = (N_s - 1) / 2) and a tone at every step's fractional k0
    the widened sum is exactly N_s per step (Parseval: sum_k |Y_k|^2 = N_s (M - 1))."""
    rng = _rng(31)
    M, n_s, L, tb = 9, 15, 8, 12
    Y = rng.normal(size=(20, n_s)) + 1j * rng.normal(size=(20, n_s))
    assert abs(cg.trajectory_widened(Y, M, n_s, 0.0, tb, 3, L, 0) - cg.trajectory(Y, M, n_s, 0.0, tb, 3, L)) < 1e-12
    k_end = 6.4
    G = np.zeros((tb, M - 1), dtype=complex)
    for m in range(tb):
        k0 = k_end * (m * L + (L - 1) / 2.0) / (tb * L)
        G[m] = np.exp(2j * np.pi * np.arange(1, M) * k0 / n_s)
    Yt = cg.spatial_dft(G, n_s)
    P = cg.trajectory_widened(Yt, M, n_s, k_end, tb, 0, L, (n_s - 1) // 2)
    assert abs(P - n_s * tb) < 1e-9 * n_s * tb
    # and the widened sum recovers more of a between-bin tone than the single bin
    assert abs(cg.trajectory_widened(Yt, M, n_s, k_end, tb, 0, L, 2)) > abs(cg.trajectory_widened(Yt, M, n_s, k_end,
                                                                                                  tb, 0, L, 0))


def test_sampling_rule_and_integration():
    """kappa_t = max(1, |k_end| kappa_t0) samples per trajectory: hand values; a = 1 is
    Eq. chimg_pth; integrating a blocks first and running the plain trajectory on the
    coarse blocks (length a L) is the same sum."""
    assert cg.sampling_blocks(9.0, 240, 5.0) == 5       # kappa_t = 45
    assert cg.sampling_blocks(0.0, 240, 5.0) == 240     # kappa_t = 1: one sample
    assert cg.sampling_blocks(100.0, 240, 5.0) == 1     # more samples than blocks
    rng = _rng(32)
    M, n_s, L = 8, 16, 4
    Y = rng.normal(size=(60, n_s)) + 1j * rng.normal(size=(60, n_s))
    assert abs(cg.trajectory_sampled(Y, M, n_s, 5.5, 24, 7, L, 1) - cg.trajectory(Y, M, n_s, 5.5, 24, 7, L)) < 1e-12
    a, tb, m0 = 4, 24, 7
    coarse = np.stack([Y[m0 + j * a:m0 + (j + 1) * a].sum(axis=0) for j in range(tb // a)])
    ref = cg.trajectory(coarse, M, n_s, 5.5, tb // a, 0, a * L)
    assert abs(cg.trajectory_sampled(Y, M, n_s, 5.5, tb, m0, L, a) - ref) < 1e-12


def test_sampling_keeps_coherence_at_five_samples_per_bin():
    """App. B: sampling a trajectory about five times per bin crossed (kappa_t0 = 5)
    keeps the coherence above 95 %: a chirp on a uniform line, the integrated trajectory
    against the finest one."""
    M, n_s, L, f_s = 16, 32, 8, 1e6
    tb, m0 = 240, 4
    for k_end in (3.0, 9.0):
        tau1 = k_end / (n_s * f_s)
        s = ula_chirp(M, (m0 + tb + 4) * L, f_s, tb * L, tau1, m0 * L)
        Y = cg.spatial_dft(cg.grid_blocks(s, L), n_s)
        fine = abs(cg.trajectory(Y, M, n_s, k_end, tb, m0, L))
        a = cg.sampling_blocks(k_end, tb, 5.0)
        coarse = abs(cg.trajectory_sampled(Y, M, n_s, k_end, tb, m0, L, a))
        assert a > 1 and coarse / fine > 0.95, (k_end, a, coarse / fine)


def test_planar_dft_is_the_2d_fft():
    rng = _rng(33)
    G = rng.normal(size=(2, 8, 8)) + 1j * rng.normal(size=(2, 8, 8))
    assert np.allclose(cg.spatial_dft_2d(G, 8), np.fft.fft2(G, axes=(1, 2)), atol=1e-11)


def test_planar_response_of_a_full_rectangle():
    """Cells cu = 1 .. A, cv = 0 .. B - 1: R(x) is the product of two geometric sums."""
    A, B, n_s = 5, 3, 16
    cells = {(cu, cv): [] for cu in range(1, A + 1) for cv in range(B)}
    for xu, xv in [(0.3, -0.2), (0.0, 0.45), (-0.5, 0.5)]:
        gu = sum(np.exp(2j * np.pi * xu * c / n_s) for c in range(1, A + 1))
        ru = np.exp(1j * np.pi * (A + 1) * xu / n_s) * (np.sin(np.pi * A * xu / n_s) / np.sin(np.pi * xu / n_s)
                                                        if xu else A)
        rv = np.exp(1j * np.pi * (B - 1) * xv / n_s) * (np.sin(np.pi * B * xv / n_s) / np.sin(np.pi * xv / n_s)
                                                        if xv else B)
        assert abs(gu - ru) < 1e-12
        assert abs(cg.response_2d(cells, xu, xv, n_s) - ru * rv) < 1e-11


def test_planar_functions_reduce_to_the_line():
    """Antennas on the u axis at whole spacings: cells (l, 0) carry the line's spacings,
    every kv column of the planar DFT is the line's DFT, and the planar trajectory with
    k_end = (k, 0) is Eq. chimg_pth's."""
    rng = _rng(34)
    M, n_s, L = 6, 16, 4
    s = rng.normal(size=(M, 64)) + 1j * rng.normal(size=(M, 64))
    pos = np.stack([np.arange(M) * 2.5, np.zeros(M)], axis=1)
    cells = cg.nearest_cells_2d(pos, 2.5)
    assert sorted(cells) == [(l, 0) for l in range(1, M)]
    G2 = cg.grid_blocks_2d(s, L, cells, n_s)
    G1 = cg.grid_blocks(s, L)
    assert np.allclose(G2[:, 1:M, 0], G1, atol=1e-13)
    Y2 = cg.spatial_dft_2d(G2, n_s)
    Y1 = cg.spatial_dft(G1, n_s)
    for kv in (0, 5):
        assert np.allclose(Y2[:, :, kv], Y1, atol=1e-11)
    for k_end in (3.3, -2.0):
        assert abs(cg.trajectory_2d(Y2, cells, n_s, (k_end, 0.0), 12, 2, L) - cg.trajectory(Y1, M, n_s, k_end, 12, 2,
                                                                                             L)) < 1e-10


def planar_chirp(pos, n_samp, f_s, t_samples, direction, start):
    """A chirp sweeping f_s in t_samples samples from direction cosines (l, m), reaching
    antenna p at (x, y) a time (x l + y m) / c late."""
    c = 299792458.0
    fdot = f_s * f_s / t_samples
    t = (np.arange(n_samp) - start) / f_s
    tau = (pos @ np.asarray(direction)) / c
    tp = t[None, :] - tau[:, None]
    on = (tp >= 0) & (tp < t_samples / f_s)
    return np.where(on, np.exp(1j * np.pi * fdot * tp ** 2), 0)


def test_planar_trajectory_finds_a_chirp():
    """A chirp on 12 antennas at random points of a 6 x 6 grid: the planar trajectory at
    the true end bins (k_end = N_s spacing f_s (l, m) / c), duration and start beats its
    neighbours in each of them."""
    rng = _rng(35)
    n_s, L, f_s, spacing = 32, 8, 1e6, 40.0
    pts = rng.choice(36, 12, replace=False)
    pos = np.stack([(pts % 6) * spacing, (pts // 6) * spacing], axis=1).astype(float)
    cells = cg.nearest_cells_2d(pos, spacing)
    k_end = np.array([7.0, -4.0])
    direction = k_end * 299792458.0 / (n_s * spacing * f_s)
    tb, m0 = 32, 3
    s = planar_chirp(pos, (m0 + tb + 10) * L, f_s, tb * L, direction, m0 * L)
    Y = cg.spatial_dft_2d(cg.grid_blocks_2d(s, L, cells, n_s), n_s)
    best = abs(cg.trajectory_2d(Y, cells, n_s, k_end, tb, m0, L))
    assert best > 0.8 * len(cells) * tb
    for dk in ([1, 0], [-1, 0], [0, 1], [0, -1]):
        assert abs(cg.trajectory_2d(Y, cells, n_s, k_end + np.array(dk), tb, m0, L)) < best
    for dt, dm in ((6, 0), (-6, 0), (0, 2), (0, -2)):
        assert abs(cg.trajectory_2d(Y, cells, n_s, k_end, tb + dt, m0 + dm, L)) < best


def test_widened_and_sampled_together_is_widening_the_integrated_blocks():
    """The widened sum over integrated samples equals the widened sum run on blocks
    integrated beforehand (the coarse blocks being a L samples long)."""
    rng = _rng(36)
    M, n_s, L, a, tb, m0 = 10, 32, 4, 3, 21, 5
    Y = rng.normal(size=(40, n_s)) + 1j * rng.normal(size=(40, n_s))
    coarse = np.stack([Y[m0 + j * a:m0 + (j + 1) * a].sum(axis=0) for j in range(tb // a)])
    ref = cg.trajectory_widened(coarse, M, n_s, 7.7, tb // a, 0, a * L, 2)
    assert abs(cg.trajectory_widened(Y, M, n_s, 7.7, tb, m0, L, 2, a=a) - ref) < 1e-10
