"""GPU parity of the antenna-block correlator, used above 64 antennas.

Antennas are cut into blocks of 128 and every block pair (I <= J) is one
workgroup of complex 16 x 16 MFMA tiles.  Cases: one partly filled block (65,
80), a second block with two antennas (130), two blocks with an off-diagonal
pair (200, and 256 = two full blocks), odd and even dump lengths (an odd one
makes a dump's last sample pair straddle its end), both output layouts, and the
reduced-precision inputs.  Tolerances as for the
stacked-row correlator: 1e-5 normalised for FP32, and for binary16 / E4M3 the
bounds of the precision tests.
"""
import numpy as np
import pytest

import synth
from gpu_helpers import compare_with_oracle, quant_errors, run_gpu, say

pytestmark = pytest.mark.gpu

TOL = 1e-5


def _cfg(seed, m_ant, s, dump_len, n_chan=2, n_dm=3, ci8=True):
    return synth.make_small(seed=seed, m_ant=m_ant, n_chan=n_chan, s=s, f_lo=1.2e9, f_s=1e6, n_dm=n_dm,
                            dm_max=150.0, dump_len=dump_len, ci8=ci8, n_pulses=1)


@pytest.mark.parametrize("m_ant,dump_len", [(65, 99), (80, 100), (130, 64), (200, 99), (256, 77)])
def test_block_correlator_fp32(gpu, m_ant, dump_len):
    cfg = _cfg(40 + m_ant, m_ant, 7001, dump_len)
    say("block correlator: %d antennas, L %d, ci8, 2 ch, 3 DMs" % (m_ant, dump_len))
    vis, lay = run_gpu(cfg, in_dtype="ci8")
    assert vis.shape[0] == 7001 // dump_len
    assert lay["n_baselines"] == m_ant * (m_ant + 1) // 2
    iu, ju = np.triu_indices(m_ant)
    assert np.all(vis.reshape(vis.shape[0], -1, iu.size)[..., iu == ju].imag == 0)
    err = compare_with_oracle(cfg, vis, lay)
    say("M %d max normalised error %.3e" % (m_ant, err))
    assert err <= TOL


def test_block_correlator_full_layout(gpu):
    m = 80
    cfg = _cfg(49, m, 5000, 100, n_chan=1)
    vis, lay = run_gpu(cfg, in_dtype="ci8", out_mode="full")
    full = vis.reshape(vis.shape[0], -1, m, m)
    assert np.array_equal(full, np.conj(np.swapaxes(full, -1, -2)))
    assert np.all(np.diagonal(full, axis1=-2, axis2=-1).imag == 0)
    iu, ju = np.triu_indices(m)
    packed = full[..., iu, ju].reshape(vis.shape[0], -1)
    err = compare_with_oracle(cfg, packed, dict(lay, n_baselines=iu.size))
    say("M 80 full layout max normalised error %.3e" % err)
    assert err <= TOL


@pytest.mark.parametrize("quant", ["f16", "e4m3"])
def test_block_correlator_quantised(gpu, quant):
    cfg = synth.make_small(seed=51, m_ant=96, n_chan=1, s=12000, f_lo=1.2e9, f_s=1e6, n_dm=3, dm_max=300.0,
                           dump_len=1000, ci8=True, n_pulses=1)
    say("block correlator, 96 antennas, inputs", quant)
    vis, lay = run_gpu(cfg, in_dtype="ci8", corr=quant)
    emu, exact, dm0 = quant_errors(cfg, vis, lay, quant, lay["scale"])
    say("%s: vs emulating oracle max %.2e rms %.2e; vs FP64 max %.2e; DM 0 max %.2e"
        % (quant, emu.max(), np.sqrt(np.mean(emu ** 2)), exact.max(), dm0.max()))
    if quant == "f16":
        assert float(np.mean(emu > 1e-5)) <= 0.01 and emu.max() <= 1e-4
    else:
        assert np.sqrt(np.mean(emu ** 2)) <= 2e-4 and emu.max() <= 5e-3
    assert exact.max() <= (1e-2 if quant == "e4m3" else 1e-4)
    assert dm0.max() <= (1e-2 if quant == "e4m3" else 1e-4)
