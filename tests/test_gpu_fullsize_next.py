"""Parity at the benchmark sizes of the next rows, on sampled outputs that the FP64
oracle computes one by one: the Chirpolator pre-integrator (36 antennas, 2^22
samples, N 2^16, L 1024, bins -100..100), the image on its output (65 536
directions, F = 2, one image per 16 windows), incoherent dedispersion (1024
channels x 2^18 samples, 1024 trials, brute force and tree) and the Chimageator
(64-antenna line, 2^22 samples, L 64, 128 bins, 256 trials), each in the launch
configuration bench.py times."""
import numpy as np
import pytest
import torch

from gpu_helpers import say
from oracle import chimageator as ocg
from oracle import chirpolator as och
from oracle import imaging as oim
from oracle import incoherent as oinc
import synth

pytestmark = pytest.mark.gpu


def test_preintegrator_and_image_at_bench_size(gpu):
    from paper_1109_3186_amd import Chirp, Image
    dev = torch.device("cuda:0")
    M, n, N, L, kmax = 36, 1 << 22, 1 << 16, 1024, 100
    g = torch.Generator(device=dev)
    g.manual_seed(1109)
    volts = torch.randn((M, n), dtype=torch.complex64, device=dev, generator=g)
    with Chirp(M, N, L, kmax, max_samples=n) as c:
        out = c.preintegrate(volts)
    torch.cuda.synchronize()
    rng = np.random.Generator(np.random.PCG64(900))
    pairs = och.pairs(M)
    worst = 0.0
    for _ in range(6):
        b = int(rng.integers(len(pairs)))
        p, q = pairs[b]
        w = int(rng.integers(out.shape[0]))
        x = och.mix(volts[[p, q]].cpu().numpy(), 0, 1)
        got = out[w, b].cpu().numpy()
        for j in rng.integers(0, 2 * kmax + 1, 4):
            ref = och.window_dft(x, w * L + N, N, int(j) - kmax)
            worst = max(worst, abs(got[j] - ref) / np.sqrt(2.0 * N))
    say("pre-integrator at bench size: max error / sqrt(2 N) %.3e" % worst)
    assert worst <= 1e-5

    # the image of the same output, as bench.py makes it
    F, lmax, w_step, f_s = 2, 0.01, 16, 1e6
    pos = synth.antenna_positions(np.random.Generator(np.random.PCG64(36)), M, 3000.0)
    heights = np.random.Generator(np.random.PCG64(37)).uniform(-20.0, 20.0, M)
    ant = np.concatenate([pos, heights[:, None]], axis=1)
    b_max = max(np.linalg.norm(ant[i] - ant[j]) for i in range(M) for j in range(i + 1, M))
    fdot = (kmax - F) * f_s * 299792458.0 / (N * b_max * lmax * np.sqrt(2.0))
    pix = synth.direction_grid(lmax, 256)
    with Image(ant, pix, fdot, f_s, N, L, kmax, F) as h:
        P, _ = h.run(out, w_step=w_step, want_e=False)
    torch.cuda.synchronize()
    scale = np.sqrt(len(pairs) * (2 * F + 1) * 2.0 * N)
    worst = 0.0
    for _ in range(3):
        img = int(rng.integers(P.shape[0]))
        sel = rng.integers(0, pix.shape[0], 6)
        rows = out[img * w_step:img * w_step + 1].cpu().numpy()
        ref = oim.image(rows, ant, pix[sel], fdot, f_s, N, L, kmax, F, first_window=img * w_step)
        got = P[img, torch.as_tensor(sel, device=dev)].cpu().numpy()
        worst = max(worst, np.max(np.abs(got - ref[0])) / scale)
    say("image at bench size: max error / (sqrt(pairs taps) bin rms) %.3e" % worst)
    assert worst <= 1e-5


def test_incoherent_at_bench_size(gpu):
    from paper_1109_3186_amd import incoherent_dedisperse, incoherent_delays, tree_dedisperse
    dev = torch.device("cuda:0")
    C, T, D, k_dm = 1024, 1 << 18, 1024, 4.148808e15
    f = 1.5e9 - (0.3e9 / C) * (np.arange(C) + 0.5)
    dms = np.linspace(0.0, 1000.0, D)
    t_samp = k_dm * 1000.0 * (1.0 / f.min() ** 2 - 1.0 / f.max() ** 2) / 1023.0
    dl = incoherent_delays(f, t_samp, dms, k_dm)
    g = torch.Generator(device=dev)
    g.manual_seed(1113)
    power = torch.rand((C, T), dtype=torch.float32, device=dev, generator=g)
    n_out = T - int(dl.max())
    brute = incoherent_dedisperse(power, torch.from_numpy(dl).to(dev), n_out)
    tree = tree_dedisperse(power)
    torch.cuda.synchronize()
    rng = np.random.Generator(np.random.PCG64(901))
    chans = torch.arange(C, device=dev)
    worst_b = worst_t = 0.0
    for _ in range(8):
        d, t = int(rng.integers(D)), int(rng.integers(n_out))
        ref = power[chans, torch.from_numpy(t + dl[:, d]).to(dev)].double().sum().item()
        worst_b = max(worst_b, abs(brute[d, t].item() - ref) / C)
        j, t = int(rng.integers(C)), int(rng.integers(T - C))
        idx = torch.as_tensor(t + np.array(oinc.tree_delays(C, j)), device=dev)
        ref = power[chans, idx].double().sum().item()
        worst_t = max(worst_t, abs(tree[j, t].item() - ref) / C)
    say("incoherent at bench size: brute max error / C %.3e, tree %.3e" % (worst_b, worst_t))
    assert worst_b <= 1e-6 and worst_t <= 1e-6


def test_chimageator_at_bench_size(gpu):
    from paper_1109_3186_amd import chimg_preintegrate, chimg_trajectories
    dev = torch.device("cuda:0")
    M, n, L, n_s = 64, 1 << 22, 64, 128
    g = torch.Generator(device=dev)
    g.manual_seed(1114)
    volts = torch.randn((M, n), dtype=torch.complex64, device=dev, generator=g)
    y = chimg_preintegrate(volts, L, n_s)
    trials = [(float(ke), tb) for tb in (64, 128, 256, 512) for ke in range(-32, 32)]
    P = chimg_trajectories(y, M, L, [t[0] for t in trials], [t[1] for t in trials])
    torch.cuda.synchronize()
    rng = np.random.Generator(np.random.PCG64(902))
    worst = 0.0
    for m in rng.integers(0, n // L, 5):
        s = volts[:, int(m) * L:(int(m) + 1) * L].cpu().numpy()
        ref = ocg.spatial_dft(ocg.grid_blocks(s, L), n_s)[0]
        got = y[:, int(m)].cpu().numpy()
        worst = max(worst, np.max(np.abs(got - ref)) / np.sqrt(np.mean(np.abs(ref) ** 2)))
    say("chimageator pre at bench size: max error / rms %.3e" % worst)
    assert worst <= 1e-5
    yh = y.cpu().numpy().T                       # [blocks][bins] for the oracle
    worst = 0.0
    for _ in range(6):
        i = int(rng.integers(len(trials)))
        ke, tb = trials[i]
        m0 = int(rng.integers(0, n // L - tb + 1))
        ref = ocg.trajectory(yh, M, n_s, ke, tb, m0, L)
        worst = max(worst, abs(P[i, m0].item() - ref) / np.sqrt(tb))
    say("chimageator trajectories at bench size: max error / sqrt(T) %.3e" % worst)
    assert worst <= 1e-5
