"""GPU parity of the Chimageator on a uniform linear array (ddx_chimg_*, Sec. 4)
against the FP64 oracle (oracle/chimageator.py): the pre-integrator (gridding,
block integration, spatial DFT) for natural and uniform weights, antenna counts up
to the 257 limit, blocks longer than one LDS round; the trajectory sums for ragged
trial sets and starts near the end; and end to end, a chirp on the array found at
its slope, end bin and start.  Bound: FP32 sums -> 1e-5 of the outputs' scale."""
import numpy as np
import pytest
import torch

from gpu_helpers import say
from oracle import chimageator as ocg
from paper_1109_3186_amd import chimg_preintegrate, chimg_trajectories
import synth

pytestmark = pytest.mark.gpu


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a.astype(np.complex64))).to("cuda:0")


@pytest.mark.parametrize("M,L,n_s,extra,natural", [(8, 16, 16, 5, True), (33, 40, 64, 0, False),
                                                   (257, 24, 256, 3, True), (16, 700, 32, 11, True)])
def test_preintegrator_matches_oracle(gpu, M, L, n_s, extra, natural):
    s = synth.noise_complex(np.random.Generator(np.random.PCG64(800 + M)), (M, 7 * L + extra))
    say("chimageator pre: M %d L %d N_s %d" % (M, L, n_s))
    got = chimg_preintegrate(_dev(s), L, n_s, natural).cpu().numpy().T
    ref = ocg.spatial_dft(ocg.grid_blocks(s, L, "natural" if natural else "uniform"), n_s)
    assert got.shape == ref.shape
    err = np.max(np.abs(got - ref)) / np.sqrt(np.mean(np.abs(ref) ** 2))
    say("max error / rms %.3e" % err)
    assert err <= 1e-5


def test_trajectories_match_oracle(gpu):
    rng = np.random.Generator(np.random.PCG64(810))
    M, n_s, L, nb = 12, 32, 8, 60
    Y = synth.noise_complex(rng, (nb, n_s))
    trials = [(9.0, 24), (5.3, 40), (-3.7, 7), (31.2, 60), (0.0, 1), (12.5, 61)]
    got = chimg_trajectories(_dev(Y.T), M, L, [t[0] for t in trials], [t[1] for t in trials]).cpu().numpy()
    ref = ocg.trajectories(Y, M, n_s, trials, L)
    err = np.max(np.abs(got - ref)) / np.sqrt(max(t[1] for t in trials))
    say("trajectories: max error / sqrt(T) %.3e" % err)
    assert err <= 1e-5
    assert np.all(got[5] == 0)        # the 61-block trial fits nowhere in 60 blocks


def test_chirp_found_end_to_end(gpu):
    import test_oracle_chimageator as toc
    M, n_s, L, f_s = 16, 32, 16, 1e6
    tb, m0, k_end = 24, 5, 9.0
    tau1 = k_end / (n_s * f_s)
    s = toc.ula_chirp(M, (m0 + tb + 6) * L, f_s, tb * L, tau1, m0 * L)
    y = chimg_preintegrate(_dev(s), L, n_s)
    trials = [(k_end + dk, tb + dt) for dk in (-1.0, 0.0, 1.0) for dt in (-6, 0, 6)]
    P = np.abs(chimg_trajectories(y, M, L, [t[0] for t in trials], [t[1] for t in trials]).cpu().numpy())
    i, m = np.unravel_index(np.argmax(P), P.shape)
    say("best trial %s at block %d: |P| %.1f of %d" % (trials[i], m, P[i, m], (M - 1) * tb))
    assert trials[i] == (k_end, tb) and m == m0 and P[i, m] > 0.85 * (M - 1) * tb


def test_long_trajectories_span_several_step_tables(gpu):
    """Trials longer than one LDS table of steps (1024): the steps are made in
    rounds."""
    rng = np.random.Generator(np.random.PCG64(820))
    M, n_s, L, nb = 8, 16, 4, 1100
    Y = synth.noise_complex(rng, (nb, n_s))
    trials = [(7.7, 1050), (-5.0, 1025)]
    got = chimg_trajectories(_dev(Y.T), M, L, [t[0] for t in trials], [t[1] for t in trials]).cpu().numpy()
    ref = ocg.trajectories(Y, M, n_s, trials, L)
    err = np.max(np.abs(got - ref)) / np.sqrt(1050)
    say("long trajectories: max error / sqrt(T) %.3e" % err)
    assert err <= 1e-5


def test_gradient_sums_match_oracle(gpu):
    """App. B partial sums: every duration of a common-gradient line from one pass,
    including durations past one step table and past the end of the blocks."""
    from paper_1109_3186_amd import chimg_gradient_sums
    rng = np.random.Generator(np.random.PCG64(830))
    M, n_s, L, nb = 10, 32, 8, 1100
    Y = synth.noise_complex(rng, (nb, n_s))
    grads, lengths = [0.37, -0.81, 0.0], [1, 3, 3, 40, 1030, 1200]
    got = chimg_gradient_sums(_dev(Y.T), M, L, grads, lengths).cpu().numpy()
    ref = ocg.gradient_sums(Y, M, n_s, grads, lengths[:4], L)
    err = np.max(np.abs(got[:, :4] - ref)) / np.sqrt(40)
    say("gradient sums (short): max error / sqrt(T) %.3e" % err)
    assert err <= 1e-5
    for i, g in enumerate(grads):             # the long duration against the trajectory form
        for m0 in (0, 33, nb - 1030):
            r = ocg.trajectory(Y, M, n_s, g * 1030, 1030, m0, L)
            assert abs(got[i, 4, m0] - r) / np.sqrt(1030) <= 1e-5
    assert np.all(got[:, 5] == 0)             # 1200 blocks fit nowhere in 1100


def test_cell_gridding_matches_oracle(gpu):
    """Gridding onto cells: a uniform line reproduces the spacing path; a sparse,
    jittered line matches the oracle's cell gridding, and the chirp on it is found
    end to end (trajectories over the cells as a line of n_cells + 1 elements)."""
    from paper_1109_3186_amd import chimg_cells, chimg_preintegrate_cells
    rng = np.random.Generator(np.random.PCG64(840))
    M, L, n_s = 9, 16, 32
    s = synth.noise_complex(rng, (M, 6 * L + 3))
    ptr, prs = chimg_cells(np.arange(M) * 40.0, 40.0, M - 1)
    got = chimg_preintegrate_cells(_dev(s), L, n_s, ptr, prs).cpu().numpy()
    spc = chimg_preintegrate(_dev(s), L, n_s).cpu().numpy()
    assert np.max(np.abs(got - spc)) <= 1e-5 * np.sqrt(np.mean(np.abs(spc) ** 2))

    pos_idx = np.array([0, 1, 3, 4, 7, 8, 11, 15, 16, 20])
    x = pos_idx * 30.0 + rng.uniform(-4, 4, pos_idx.size)
    ptr, prs = chimg_cells(x, 30.0, 20)
    s = synth.noise_complex(rng, (pos_idx.size, 5 * L))
    got = chimg_preintegrate_cells(_dev(s), L, 64, ptr, prs).cpu().numpy().T
    ref = ocg.spatial_dft(ocg.grid_blocks_cells(s, L, ocg.nearest_cells(x, 30.0), 20), 64)
    err = np.max(np.abs(got - ref)) / np.sqrt(np.mean(np.abs(ref) ** 2))
    say("cell gridding: max error / rms %.3e" % err)
    assert err <= 1e-5

    M2, n_s2, L2, f_s = 10, 64, 16, 1e6
    tb, m0, k_end = 20, 4, 11.0
    tau1 = k_end / (n_s2 * f_s)
    fdot = f_s * f_s / (tb * L2)
    t = (np.arange((m0 + tb + 6) * L2) - m0 * L2) / f_s
    tp = t[None, :] - (pos_idx * tau1)[:, None]
    sc = np.where((tp >= 0) & (tp < tb * L2 / f_s), np.exp(1j * np.pi * fdot * tp ** 2), 0)
    ptr, prs = chimg_cells(pos_idx * 30.0, 30.0, 20)
    y = chimg_preintegrate_cells(_dev(sc), L2, n_s2, ptr, prs)
    trials = [(k_end + dk, tb + dt) for dk in (-1.0, 0.0, 1.0) for dt in (-5, 0, 5)]
    P = np.abs(chimg_trajectories(y, 21, L2, [t_[0] for t_ in trials], [t_[1] for t_ in trials]).cpu().numpy())
    i, m = np.unravel_index(np.argmax(P), P.shape)
    say("sparse line: best trial %s at block %d" % (trials[i], m))
    assert trials[i] == (k_end, tb) and m == m0


# ---- App. B: widened and sampled trajectories; planar gridding and trajectories ----


def _traj_ref(Y, M, n_s, trials, L, F, a_list):
    nb = Y.shape[0]
    P = np.zeros((len(trials), nb), dtype=np.complex128)
    for i, ((k_end, tb), a) in enumerate(zip(trials, a_list)):
        for m0 in range(0, nb - tb + 1):
            if F == 0:
                P[i, m0] = ocg.trajectory_sampled(Y, M, n_s, k_end, tb, m0, L, a)
            else:
                P[i, m0] = ocg.trajectory_widened(Y, M, n_s, k_end, tb, m0, L, F, a=a)
    return P


@pytest.mark.parametrize("F,sampled", [(0, True), (2, False), (3, True), (8, False)])
def test_widened_sampled_trajectories_match_oracle(gpu, F, sampled):
    from paper_1109_3186_amd import chimg_trajectories_ext
    rng = np.random.Generator(np.random.PCG64(820 + F))
    M, n_s, L, nb = 12, 32, 8, 70
    Y = synth.noise_complex(rng, (nb, n_s))
    trials = [(9.0, 24), (5.3, 40), (-3.7, 7), (31.2, 60), (0.0, 1), (12.5, 71), (2.2, 30)]
    a_list = [3, 4, 2, 7, 1, 1, 30] if sampled else [1] * len(trials)
    say("widened/sampled trajectories: F %d, a %s" % (F, a_list))
    got = chimg_trajectories_ext(_dev(Y.T), M, L, [t[0] for t in trials], [t[1] for t in trials],
                                 a_blocks=a_list if sampled else None, half_width=F).cpu().numpy()
    ref = _traj_ref(Y, M, n_s, trials, L, F, a_list)
    err = np.max(np.abs(got - ref)) / np.sqrt(max(t[1] for t in trials) * (2 * F + 1))
    say("max error / sqrt(T (2F + 1)) %.3e" % err)
    assert err <= 1e-5
    assert np.all(got[5] == 0)        # the 71-block trial fits nowhere in 70 blocks


def test_sampling_rule_matches_oracle(gpu):
    from paper_1109_3186_amd import chimg_sampling_blocks
    for k_end, tb, kap in [(9.0, 240, 5.0), (0.0, 240, 5.0), (100.0, 240, 5.0), (-3.3, 77, 2.5), (7.0, 7, 0.0)]:
        assert chimg_sampling_blocks(k_end, tb, kap) == ocg.sampling_blocks(k_end, tb, kap)


def _planar_array(seed, m_ant, side, spacing):
    rng = np.random.Generator(np.random.PCG64(seed))
    pts = rng.choice(side * side, m_ant, replace=False)
    return np.stack([(pts % side) * spacing, (pts // side) * spacing], axis=1).astype(float)


def _cells_from_lib(pos, spacing):
    from paper_1109_3186_amd import chimg_cells_2d
    ptr, pairs, uv = chimg_cells_2d(pos, spacing)
    cells = {}
    for c in range(uv.shape[0]):
        cells[(int(uv[c, 0]), int(uv[c, 1]))] = [tuple(int(v) for v in pairs[b]) for b in range(ptr[c], ptr[c + 1])]
    return (ptr, pairs, uv), cells


def test_planar_cells_match_oracle(gpu):
    for seed, m, jitter in [(830, 12, 0.0), (831, 40, 7.0), (832, 64, 19.9)]:
        pos = _planar_array(seed, m, 9, 40.0) + np.random.Generator(np.random.PCG64(seed)).uniform(-jitter, jitter,
                                                                                                  (m, 2))
        _, cells = _cells_from_lib(pos, 40.0)
        ref = ocg.nearest_cells_2d(pos, 40.0)
        assert cells == {k: ref[k] for k in sorted(ref)}
        assert list(cells) == sorted(ref)


@pytest.mark.parametrize("m_ant,n_s,L,extra", [(12, 16, 16, 3), (40, 32, 24, 0), (64, 64, 100, 7)])
def test_planar_preintegrator_matches_oracle(gpu, m_ant, n_s, L, extra):
    from paper_1109_3186_amd import chimg_preintegrate_2d
    pos = _planar_array(840 + m_ant, m_ant, 8, 25.0)
    tables, cells = _cells_from_lib(pos, 25.0)
    s = synth.noise_complex(np.random.Generator(np.random.PCG64(850 + m_ant)), (m_ant, 6 * L + extra))
    say("planar pre: M %d, %d cells, N_s %d, L %d" % (m_ant, len(cells), n_s, L))
    got = chimg_preintegrate_2d(_dev(s), L, n_s, tables).cpu().numpy().T.reshape(-1, n_s, n_s)
    ref = ocg.spatial_dft_2d(ocg.grid_blocks_2d(s, L, cells, n_s), n_s)
    err = np.max(np.abs(got - ref)) / np.sqrt(np.mean(np.abs(ref) ** 2))
    say("max error / rms %.3e" % err)
    assert err <= 1e-5


def test_planar_trajectories_match_oracle_and_find_a_chirp(gpu):
    import test_oracle_chimageator as toc

    from paper_1109_3186_amd import chimg_preintegrate_2d, chimg_trajectories_2d
    n_s, L, f_s, spacing = 32, 8, 1e6, 40.0
    pos = _planar_array(35, 12, 6, spacing)
    tables, cells = _cells_from_lib(pos, spacing)
    k_end = np.array([7.0, -4.0])
    direction = k_end * 299792458.0 / (n_s * spacing * f_s)
    tb, m0 = 32, 3
    s = toc.planar_chirp(pos, (m0 + tb + 10) * L, f_s, tb * L, direction, m0 * L)
    rng = np.random.Generator(np.random.PCG64(860))
    s = s + 0.3 * synth.noise_complex(rng, s.shape)
    # parity on the oracle's own pre-integrator output (the same input on both sides)
    Y = ocg.spatial_dft_2d(ocg.grid_blocks_2d(s, L, cells, n_s), n_s)
    y_ref = _dev(Y.reshape(Y.shape[0], -1).T)
    trials = [(k_end + np.array(dk, float), tb + dt) for dk in ([0, 0], [1, 0], [0, -1], [-1, 1]) for dt in (0, 6)]
    trials.append((np.array([2.6, 3.4]), 5))
    P = chimg_trajectories_2d(y_ref, n_s, L, tables[2], [t[0] for t in trials], [t[1] for t in trials]).cpu().numpy()
    nb = Y.shape[0]
    worst = 0.0
    for i, (ke, t) in enumerate(trials):
        for m in range(nb):
            ref = ocg.trajectory_2d(Y, cells, n_s, ke, t, m, L) if m + t <= nb else 0.0
            worst = max(worst, abs(P[i, m] - ref))
    # every term is at most max|Y| (the chirp's bins are ~ the cell count, far above the
    # noise): the error scale of a T-term FP32 sum is max|Y| sqrt(T)
    scale = np.max(np.abs(Y)) * np.sqrt(max(t for _, t in trials))
    say("planar trajectories: max error / (max|Y| sqrt(T)) %.3e" % (worst / scale))
    assert worst <= 1e-5 * scale
    # end to end on the device: the GPU pre-integrator, then the GPU trajectories
    y = chimg_preintegrate_2d(_dev(s), L, n_s, tables)
    P = np.abs(chimg_trajectories_2d(y, n_s, L, tables[2], [t[0] for t in trials], [t[1] for t in trials])
               .cpu().numpy())
    i, m = np.unravel_index(np.argmax(P), P.shape)
    say("best trial %s at block %d: |P| %.1f of %d" % (trials[i], m, P[i, m], len(cells) * tb))
    assert i == 0 and m == m0 and P[i, m] > 0.7 * len(cells) * tb
