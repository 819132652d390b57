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
