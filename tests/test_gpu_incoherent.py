"""GPU parity of classical incoherent dedispersion (ddx_power_beam,
ddx_incoherent_dedisperse, ddx_tree_dedisperse; Sec. 2.3.1, 2.4.1) against the
FP64 oracle (oracle/incoherent.py).  The tree is checked bit for bit on integer
power (every partial sum is exact in FP32), for channel counts below, at and above
the 32-channel group fused in LDS, sample counts that are not a multiple of the
224-sample tile, and an odd and even number of later stages.  The brute force and
the power beam are FP32 sums: held to 1e-6 of the sums' scale."""
import numpy as np
import pytest
import torch

from gpu_helpers import say
from oracle import incoherent as oinc
from paper_1109_3186_amd import incoherent_dedisperse, incoherent_delays, power_beam, tree_dedisperse
import synth

pytestmark = pytest.mark.gpu


def _dev(a, dtype):
    return torch.from_numpy(np.ascontiguousarray(a).astype(dtype)).to("cuda:0")


@pytest.mark.parametrize("C,T", [(1, 300), (2, 257), (4, 1000), (16, 513), (32, 700), (64, 1000), (128, 300),
                                 (256, 1100), (512, 700), (2048, 1500), (1024, 4100), (256, 90), (1024, 300)])
def test_tree_is_exact_on_integer_power(gpu, C, T):
    """Every mix of later passes (one, two and three stages: 64 .. 2048 channels),
    and fewer samples than the largest sweep shift."""
    p = np.random.Generator(np.random.PCG64(500 + C)).integers(0, 64, (C, T)).astype(np.float64)
    say("tree: C %d T %d" % (C, T))
    got = tree_dedisperse(_dev(p, np.float32)).cpu().numpy()
    torch.cuda.synchronize()
    assert np.array_equal(got, oinc.tree(p))


def test_tree_recovers_an_impulse_on_a_sweep(gpu):
    C, T, j0, t0 = 256, 2000, 173, 900
    p = np.zeros((C, T))
    p[np.arange(C), t0 + np.array(oinc.tree_delays(C, j0))] = 1.0
    got = tree_dedisperse(_dev(p, np.float32)).cpu().numpy()
    assert got[j0, t0] == C and got.max() == C


@pytest.mark.parametrize("C,D,extra,cut", [(48, 37, 700, True), (7, 5, 300, False), (256, 64, 1000, True)])
def test_brute_force_matches_oracle(gpu, C, D, extra, cut):
    """T = the largest delay + extra; cut: only outputs whose every sample exists,
    else all T outputs (the later ones sum zeros past the end)."""
    rng = np.random.Generator(np.random.PCG64(600 + C))
    f = 1.2e9 + 1e6 * np.arange(C)[::-1]
    dms = np.sort(rng.uniform(0, 800, D))
    dl = incoherent_delays(f, 1e-4, dms)
    assert np.array_equal(dl, oinc.dm_delays(f, 1e-4, dms))
    T = int(dl.max()) + extra
    n_out = T - int(dl.max()) if cut else T
    p = rng.random((C, T))
    say("brute force: C %d D %d T %d n_out %d" % (C, D, T, n_out))
    got = incoherent_dedisperse(_dev(p, np.float32), _dev(dl, np.int32), n_out).cpu().numpy()
    ref = oinc.brute_force(p, dl, n_out)
    err = np.max(np.abs(got - ref)) / C
    say("max error / C %.3e" % err)
    assert err <= 1e-6


@pytest.mark.parametrize("C,D,T,n_out,extreme", [(40, 70, 900, 1200, False), (9, 33, 2000, 1100, False),
                                                 (12, 40, 700, 700, True)])
def test_brute_force_any_delays(gpu, C, D, T, n_out, extreme):
    """Delays before the first sample and past the last, and channels whose delays
    spread beyond the staged span (read from global memory) next to staged ones;
    extreme: delays near +-2^30, spreads that overflow 32-bit byte offsets."""
    rng = np.random.Generator(np.random.PCG64(610 + C))
    dl = rng.integers(-400, 400, (C, D)).astype(np.int32)
    dl[::3] = rng.integers(-40, 40, (len(dl[::3]), D))      # narrow channels: staged
    if extreme:
        dl[1::3] = np.where(rng.random((len(dl[1::3]), D)) < 0.5, -1, 1) * (1 << 30) + dl[1::3]
        dl[2, :5] = [0, 2 ** 31 - 1, -2 ** 31, 5, -7]
    p = rng.random((C, T))
    say("brute force, any delays: C %d D %d T %d n_out %d" % (C, D, T, n_out))
    got = incoherent_dedisperse(_dev(p, np.float32), _dev(dl, np.int32), n_out).cpu().numpy()
    ref = oinc.brute_force(p, dl, n_out)
    assert np.max(np.abs(got - ref)) / C <= 1e-6


def test_brute_force_recovers_a_dispersed_impulse(gpu):
    C, D = 64, 33
    f = 1.2005e9 + 1e6 * np.arange(C)[::-1]
    dms = np.linspace(0, 2000, D)
    dl = incoherent_delays(f, 1e-3, dms)
    T = int(dl.max()) + 500
    p = np.zeros((C, T))
    d0, t0 = 21, 300
    p[np.arange(C), t0 + dl[:, d0]] = 1.0
    got = incoherent_dedisperse(_dev(p, np.float32), _dev(dl, np.int32), 500).cpu().numpy()
    assert got[d0, t0] == C and got.max() == C


def test_power_beam_matches_oracle(gpu):
    v = synth.noise_complex(np.random.Generator(np.random.PCG64(700)), (3, 5, 1003))
    got = power_beam(_dev(v, np.complex64), 7).cpu().numpy()
    ref = oinc.power_beam(v, 7)
    assert got.shape == ref.shape
    err = np.max(np.abs(got - ref) / ref)
    say("power beam: max relative error %.3e" % err)
    assert err <= 1e-6
