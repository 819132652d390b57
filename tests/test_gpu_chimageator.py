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
