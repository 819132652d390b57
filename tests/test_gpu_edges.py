"""Edge cases of the HIP path: lower sideband, one antenna, the largest array,
odd dump lengths in the stacked correlator, one-sample dumps, empty calls, NaN input, and the error statuses that need a
device (ring full, fetch buffer too small, device-memory cap).  Parity bar as in
test_gpu_parity: 1e-5 normalised against the FP64 oracle."""
import ctypes as ct

import numpy as np
import pytest

import synth
from gpu_helpers import compare_with_oracle, run_gpu, say, select

pytestmark = pytest.mark.gpu

TOL = 1e-5


def test_lower_sideband(gpu):
    cfg = synth.make_small(seed=80, m_ant=4, n_chan=2, s=20000, f_lo=1.3e9, f_s=1e6, n_dm=4, dm_max=300.0,
                           dump_len=100, n_pulses=1)
    vis, lay = run_gpu(cfg, sideband=-1)
    assert lay["sideband"] == -1
    err = compare_with_oracle(cfg, vis, lay)
    say("sideband -1: max normalised error %.3e" % err)
    assert err <= TOL
    up, _ = run_gpu(cfg)
    assert not np.array_equal(up, vis)  # the chirp is mirrored in frequency


def test_single_antenna(gpu):
    cfg = synth.make_small(seed=81, m_ant=1, n_chan=2, s=9000, f_lo=1.3e9, f_s=1e6, n_dm=3, dm_max=200.0,
                           dump_len=64, ci8=True, n_pulses=0)
    vis, lay = run_gpu(cfg, in_dtype="ci8")
    assert lay["n_baselines"] == 1 and np.all(vis.imag == 0) and np.all(vis.real > 0)
    assert compare_with_oracle(cfg, vis, lay) <= TOL


def test_largest_array(gpu):
    cfg = synth.make_small(seed=82, m_ant=1024, n_chan=1, s=3000, f_lo=1.4e9, f_s=1e6, n_dm=2, dm_max=20.0,
                           dump_len=1000, ci8=True, n_pulses=0)
    say("1024 antennas, 3000 samples, 2 DMs")
    vis, lay = run_gpu(cfg, in_dtype="ci8")
    assert vis.shape == (3, 2 * 1024 * 1025 // 2)
    err = compare_with_oracle(cfg, vis, lay)
    say("1024 antennas: max normalised error %.3e" % err)
    assert err <= TOL


@pytest.mark.parametrize("m_ant,dump_len", [(33, 75), (64, 101)])
def test_stacked_correlator_odd_dumps(gpu, m_ant, dump_len):
    """The stacked-row correlator at a padded tile count (33 antennas: 66 of 80
    rows) and at its largest array (64), with odd dump lengths: every dump's last
    sample pair straddles the dump's end and its second sample must be read as 0."""
    cfg = synth.make_small(seed=87 + m_ant, m_ant=m_ant, n_chan=2, s=6007, f_lo=1.3e9, f_s=1e6, n_dm=3,
                           dm_max=150.0, dump_len=dump_len, ci8=True, n_pulses=1)
    vis, lay = run_gpu(cfg, in_dtype="ci8")
    assert vis.shape[0] == 6007 // dump_len
    err = compare_with_oracle(cfg, vis, lay)
    say("stacked correlator, M %d, L %d: max normalised error %.3e" % (m_ant, dump_len, err))
    assert err <= TOL


def test_one_sample_dumps(gpu):
    """L = 1: each dump is one product y_i conj(y_j), nothing averages.  A single
    sample can sit near zero, where the per-dump normalisation sqrt(V_ii V_jj)
    divides the transform's absolute FP32 error (a fraction of the block RMS) by
    almost nothing, so the error is taken against the mean autocorrelation power;
    the largest of the 18000 products is ~9x that power and carries the split-FP16
    product's ~1e-6 relative error (hi and lo roundings, the dropped lo*lo term),
    hence a bound of 3e-5 here instead of the 1e-5 of averaged dumps."""
    import oracle
    from gpu_helpers import blockings
    cfg = synth.make_small(seed=83, m_ant=3, n_chan=1, s=3000, f_lo=1.4e9, f_s=1e6, n_dm=2, dm_max=30.0,
                           dump_len=1, n_pulses=0)
    vis, lay = run_gpu(cfg)
    assert vis.shape[0] == 3000
    ref = oracle.run_oracle(cfg["volts"], cfg["chan_freqs"], 1e6, cfg["dm_lists"], 1, blockings(lay))
    iu, ju = np.triu_indices(3)
    for (c, d), v in ref.items():
        got = select(vis, lay, c, d).astype(np.complex128)
        power = float(np.mean(v[:, iu == ju].real))
        err = float(np.max(np.abs(got - v))) / power
        say("L = 1, DM %g: max |dV| / mean auto %.3e (per-dump metric %.3e)" % (
            cfg["dm_lists"][c][d], err, compare_with_oracle(cfg, vis, lay, pairs=[(c, d)])))
        assert err <= 3e-5


def test_empty_calls_change_nothing(gpu):
    import torch

    from paper_1109_3186_amd import Plan
    cfg = synth.make_small(seed=84, m_ant=3, n_chan=2, s=12000, f_lo=1.3e9, f_s=1e6, n_dm=3, dm_max=200.0,
                           dump_len=100, n_pulses=1)
    ref, lay = run_gpu(cfg)
    x = cfg["volts"]
    outs = []
    with Plan(3, cfg["chan_freqs"], 1e6, 100, max_block_samples=12000, in_dtype="cf32") as p:
        p.set_dm_trials(cfg["dm_lists"][0])
        p.process_block(None)  # nothing yet
        p.process_block(torch.from_numpy(np.ascontiguousarray(x[..., :7000])).cuda())
        p.process_block(torch.from_numpy(np.ascontiguousarray(x[..., 7000:7000])).cuda())  # zero samples
        p.process_block(torch.from_numpy(np.ascontiguousarray(x[..., 7000:])).cuda())
        _, nd, v = p.fetch()
        if nd:
            outs.append(v.cpu().numpy())
        p.process_block(None, flush=True)  # flush with no new samples
        _, nd, v = p.fetch()
        if nd:
            outs.append(v.cpu().numpy())
        torch.cuda.synchronize()
    assert np.array_equal(np.concatenate(outs), ref)


def test_nan_input_stays_local(gpu):
    cfg = synth.make_small(seed=85, m_ant=3, n_chan=1, s=20000, f_lo=1.4e9, f_s=1e6, n_dm=1, dm_max=1.0,
                           dump_len=100, n_pulses=0)
    cfg["dm_lists"] = [np.array([0.0])]
    x = cfg["volts"].copy()
    x[0, 1, 15050] = np.nan
    vis, lay = run_gpu(dict(cfg, volts=x))
    v = select(vis, lay, 0, 0)
    bad = ~np.isfinite(v).all(axis=1)
    # DM 0 passes the sample through unchanged: only its dump goes non-finite
    assert bad[150] and bad.sum() >= 1 and np.isfinite(np.delete(v, np.flatnonzero(bad), axis=0)).all()


def test_device_side_statuses(gpu):
    import torch

    import paper_1109_3186_amd as ddx
    from paper_1109_3186_amd import DdxError, Plan
    cfg = synth.make_small(seed=86, m_ant=3, n_chan=1, s=40000, f_lo=1.4e9, f_s=1e6, n_dm=2, dm_max=50.0,
                           dump_len=100, n_pulses=0)
    x = torch.from_numpy(cfg["volts"]).cuda()
    # ring of 5 dumps: a 20000-sample call completes far more
    with Plan(3, cfg["chan_freqs"], 1e6, 100, max_block_samples=40000, in_dtype="cf32", ring_dumps=5) as p:
        p.set_dm_trials(cfg["dm_lists"][0])
        with pytest.raises(DdxError) as e:
            p.process_block(x[..., :20000].contiguous())
        assert e.value.status == ddx.EFULL
    # fetch into a buffer one record too small
    with Plan(3, cfg["chan_freqs"], 1e6, 100, max_block_samples=40000, in_dtype="cf32") as p:
        p.set_dm_trials(cfg["dm_lists"][0])
        p.process_block(x, flush=True)
        lay = p.layout()
        small = torch.empty((lay["dumps_ready"] - 1, lay["record_elems"]), dtype=torch.complex64, device="cuda")
        first, need = ct.c_int64(), ct.c_int64()
        rc = ddx.lib().ddx_fetch_visibilities(p._h, ct.c_void_p(small.data_ptr()), small.numel() * 8, ct.byref(first),
                                              ct.byref(need), ct.c_void_p(torch.cuda.current_stream().cuda_stream))
        assert rc == ddx.ESIZE and need.value == lay["dumps_ready"] and first.value == 0
        _, nd, v = p.fetch()
        assert nd == 400
        torch.cuda.synchronize()
    # a device-memory cap below what the plan needs
    with Plan(3, cfg["chan_freqs"], 1e6, 100, max_block_samples=40000, in_dtype="cf32",
              max_device_bytes=1 << 20) as p:
        with pytest.raises(DdxError) as e:
            p.set_dm_trials(cfg["dm_lists"][0])
        assert e.value.status == ddx.ENOMEM


def test_f32_split_range_follows_level_changes(gpu):
    """FP32 correlator inputs whose level rises 10^4 times after the first block window
    (which set the scale), plus one sample at 10^5 sigma: the binary16 split of each
    unit is ranged from its own largest value, so nothing overflows.  Dumps of blocks
    whose windows hold one level stay within 1e-5 (normalised) of the FP64 oracle;
    dumps of the blocks whose windows straddle the 80 dB step carry the FP32
    transform's error at that dynamic range (a single-precision FFT emulation of the
    oracle gives up to 9e-5 there), held to 1e-3."""
    import oracle
    from gpu_helpers import blockings
    cfg = synth.make_small(seed=71, m_ant=4, n_chan=2, s=40000, f_lo=1.25e9, f_s=1e6, n_dm=3, dm_max=300.0,
                           dump_len=500, n_pulses=0)
    step = 12000
    x = cfg["volts"].astype(np.complex128)
    x[..., step:] *= 1e4
    x[1, 2, 30001] = (1e5 / np.sqrt(2)) * (1 + 1j)
    cfg = dict(cfg, volts=x.astype(np.complex64))
    vis, lay = run_gpu(cfg)
    assert np.all(np.isfinite(vis))
    bl = blockings(lay)
    iu, ju = np.triu_indices(4)
    clean = mixed = 0.0
    for c in range(2):
        ref = oracle.run_oracle(cfg["volts"], cfg["chan_freqs"], 1e6, cfg["dm_lists"], 500, bl, chans=[c])
        for (cc, d), v in ref.items():
            v_, n_, lead = bl[c][d]["valid"], bl[c][d]["fft_len"], bl[c][d]["lead"]  # the DM's blocking
            blk = np.arange(vis.shape[0]) * 500 // v_          # block of each dump
            straddle = (blk * v_ - lead <= step) & (step < blk * v_ - lead + n_)
            auto = v[:, iu == ju].real
            e = (np.abs(select(vis, lay, cc, d).astype(np.complex128) - v) / np.sqrt(auto[:, iu] * auto[:, ju])).max(1)
            clean = max(clean, float(e[~straddle].max()))
            mixed = max(mixed, float(e[straddle].max()))
    say("level step 1e4 and a 1e5 sigma sample: max normalised error %.3e (one-level blocks), %.3e (blocks across "
        "the step); scales %s" % (clean, mixed, lay["scale"]))
    assert clean <= 1e-5
    assert mixed <= 1e-3
