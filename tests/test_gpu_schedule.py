"""GPU tests of the batched schedule: work lists over all channels, waves of
(channel, DM, block) units, two-pass transforms above 2^15 points, channels of
different transform lengths in one plan, and compact dump records.

Parity as elsewhere (1e-5 normalised against the FP64 oracle); the schedule
itself must not change any result, so different wave sizes and DM groups are
compared bitwise.
"""
import numpy as np
import pytest

import oracle
import synth
from gpu_helpers import compare_with_oracle, run_gpu, say, select

pytestmark = pytest.mark.gpu

TOL = 1e-5


@pytest.mark.parametrize("n", [1 << 16, 1 << 17, 1 << 18])
def test_two_pass_transform_lengths(gpu, n):
    """N = 2^16..2^18 (R = 2, 4, 8 rows of 2^15), several blocks and a ragged tail."""
    cfg = synth.make_small(seed=60 + n % 97, m_ant=3, n_chan=1, s=2 * n + 12345, f_lo=1.3e9, f_s=1e6, n_dm=3,
                           dm_max=500.0, dump_len=64, n_pulses=0)
    say("two-pass N =", n)
    vis, lay = run_gpu(cfg, fft_len=n)
    assert lay["fft_len"][0] == n
    err = compare_with_oracle(cfg, vis, lay)
    say("N %d max normalised error %.3e" % (n, err))
    assert err <= TOL


@pytest.mark.parametrize("quant,L", [("e4m3", 1000), ("f16", 40)])
def test_two_pass_quantised_autocorrelations(gpu, quant, L):
    """Reduced-precision inputs at a two-pass length: the autocorrelations are the
    unrounded voltages' power (summed from the intermediate rows, including dumps
    shorter than a wave), equal to the exact oracle's within 1e-5; cross products
    within the format's bound."""
    cfg = synth.make_small(seed=66, m_ant=5, n_chan=1, s=3 * (1 << 16) + 4321, f_lo=1.3e9, f_s=1e6, n_dm=3,
                           dm_max=500.0, dump_len=L, ci8=True, n_pulses=1)
    say("two-pass N 2^16, %s inputs, L %d" % (quant, L))
    vis, lay = run_gpu(cfg, in_dtype="ci8", corr=quant, fft_len=1 << 16)
    from gpu_helpers import blockings
    bl = blockings(lay)
    ref = oracle.run_oracle(cfg["volts"], cfg["chan_freqs"], 1e6, cfg["dm_lists"], L, bl)
    iu, ju = np.triu_indices(5)
    worst_auto = worst = 0.0
    for (c, d), v in ref.items():
        got = select(vis, lay, c, d).astype(np.complex128)
        auto = v[:, iu == ju].real
        norm = np.sqrt(auto[:, iu] * auto[:, ju])
        e = np.abs(got - v) / norm
        worst_auto = max(worst_auto, float(e[:, iu == ju].max()))
        worst = max(worst, float(e.max()))
    say("%s: autos max %.2e, all max %.2e" % (quant, worst_auto, worst))
    assert worst_auto <= TOL
    assert worst <= (1e-2 if quant == "e4m3" else 1e-3 if L < 100 else 1e-4)


def test_mixed_lengths_one_plan(gpu):
    """Channels with 2^12-, 2^15- and 2^17-point blocks and uneven DM lists in one plan,
    streamed in uneven chunks."""
    cfg = synth.make_small(seed=64, m_ant=4, n_chan=3, s=300001, f_lo=0.7e9, f_s=1e6, n_dm=2, dm_max=50.0,
                           dump_len=100, ci8=True, n_pulses=1)
    cfg["dm_lists"] = [np.array([0.0, 20.0, 45.0]), np.array([500.0, 10.0]),
                       np.array([0.0, 500.0, 1200.0, 2500.0])]
    vis, lay = run_gpu(cfg, in_dtype="ci8", chunks=[70000, 1, 130000, 100000], max_block=130000,
                       dm_classes="single")
    say("lengths", lay["fft_len"], "valid", lay["valid"])
    assert list(lay["fft_len"]) == [4096, 32768, 131072]
    for c in range(3):
        ref = oracle.blocking(cfg["chan_freqs"][c], 1e6, max(cfg["dm_lists"][c]), 100)
        assert (lay["fft_len"][c], lay["valid"][c], lay["lead"][c]) == (ref["fft_len"], ref["valid"], ref["lead"])
    err = compare_with_oracle(cfg, vis, lay)
    say("mixed lengths max normalised error %.3e" % err)
    assert err <= TOL


def test_schedule_does_not_change_results(gpu):
    cfg = synth.make_small(seed=65, m_ant=5, n_chan=3, s=40000, f_lo=1.3e9, f_s=1e6, n_dm=7, dm_max=300.0,
                           dump_len=100, ci8=True, n_pulses=1)
    cfg["dm_lists"][1] = cfg["dm_lists"][1][:3]
    ref, lay = run_gpu(cfg, in_dtype="ci8")
    say("auto schedule: wave_units %d dm_group %d" % (lay["wave_units"], lay["dm_group"]))
    for wu, dg in [(1, 1), (5, 3), (16, 16), (1000, 2)]:
        got, l2 = run_gpu(cfg, in_dtype="ci8", wave_units=wu, dm_group=dg)
        assert l2["wave_units"] <= wu and l2["dm_group"] == min(dg, 7)
        assert np.array_equal(got, ref), (wu, dg)


def test_compact_records_match_full(gpu):
    cfg = synth.make_small(seed=66, m_ant=4, n_chan=2, s=25000, f_lo=1.3e9, f_s=1e6, n_dm=6, dm_max=300.0,
                           dump_len=100, n_pulses=1)
    full, lay = run_gpu(cfg)
    mask = [np.array([0, 1, 0, 0, 1, 1], np.uint8), np.array([1, 0, 0, 0, 0, 0], np.uint8)]
    comp, lc = run_gpu(cfg, mask=mask, compact_records=True, max_record_pairs=4)
    assert lc["record_pairs"] == 4 and comp.shape[1] == 4 * lc["n_baselines"]
    pos = lc["record_pos"]
    assert list(pos) == [-1, 0, -1, -1, 1, 2, 3, -1, -1, -1, -1, -1]
    for c in range(2):
        for d in range(6):
            if mask[c][d]:
                assert np.array_equal(select(comp, lc, c, d), select(full, lay, c, d))


def test_compact_records_state_rules(gpu):
    import torch

    from paper_1109_3186_amd import DdxError, Plan
    cfg = synth.make_small(seed=67, m_ant=3, n_chan=2, s=20000, f_lo=1.3e9, f_s=1e6, n_dm=4, dm_max=200.0,
                           dump_len=100, n_pulses=0)
    with Plan(3, cfg["chan_freqs"], 1e6, 100, max_block_samples=20000, in_dtype="cf32", compact_records=True,
              max_record_pairs=3) as p:
        p.set_dm_trials(cfg["dm_lists"][0])
        lay = p.layout()
        assert lay["record_pairs"] == 0  # 8 pairs exceed the capacity: nothing active until chosen
        with pytest.raises(DdxError):
            p.set_active_dms(np.ones(4, np.uint8), chan=0)  # 4 > 3
        p.set_active_dms(np.array([1, 0, 1, 0], np.uint8), chan=0)
        p.set_active_dms(np.array([0, 0, 0, 1], np.uint8), chan=1)
        assert p.layout()["record_pairs"] == 3
        x = torch.from_numpy(cfg["volts"][:, :, :10000].copy()).cuda()
        p.process_block(x)
        torch.cuda.synchronize()
        if p.layout()["dumps_ready"] > 0:
            with pytest.raises(DdxError):
                p.set_active_dms(np.array([0, 0, 0, 0], np.uint8), chan=1)  # unfetched dumps
        p.fetch()
        torch.cuda.synchronize()
        with pytest.raises(DdxError):
            p.set_active_dms(np.array([0, 0, 1, 1], np.uint8), chan=1)  # 2 + 2 > 3
        p.set_active_dms(np.array([0, 1, 0, 0], np.uint8), chan=1)
        lay = p.layout()
        assert lay["record_pairs"] == 3 and list(lay["record_pos"]) == [0, -1, 1, -1, -1, 2, -1, -1]


def test_c3_shape_sampled(gpu):
    """256 antennas at 0.7 GHz with per-channel DM grids up to 3000 (two-pass 2^18 and
    2^17 blocks, antenna-block correlator), sampled (channel, DM) pairs against the oracle."""
    p3 = synth.c3_params()
    cfg = synth.make_small(seed=68, m_ant=256, n_chan=2, s=200000, f_lo=p3["f_lo"], f_s=1e6, n_dm=3,
                           dm_max=3000.0, dump_len=1000, ci8=True, n_pulses=1, radius_m=2500.0)
    cfg["dm_lists"] = [np.array([0.0, 750.0, 1500.0, 2250.0, 2990.0]), np.arange(3) * 3000.0 / 3]
    say("C3 shape: 256 ant, 2 ch at 0.7 GHz, 200000 ci8 samples, DMs 5 + 3 up to 2990")
    vis, lay = run_gpu(cfg, in_dtype="ci8", dm_classes="single")
    say("lengths", lay["fft_len"], "valid", lay["valid"], "dumps", vis.shape[0])
    assert list(lay["fft_len"]) == [1 << 18, 1 << 17]
    assert vis.shape[0] == 200
    err = compare_with_oracle(cfg, vis, lay, pairs=[(0, 4), (1, 1)])
    say("C3 shape max normalised error %.3e" % err)
    assert err <= TOL


def test_dm_classes_match_oracle_and_split_invariance(gpu):
    """Automatic blocking classes: low DMs take shorter transforms with less overlap.
    Every DM's blocking is the oracle's rule at its class's largest DM and the
    class's length; every (channel, DM) matches the oracle run with its own
    blocking; the classes' different block lengths give the same records however
    the stream is cut into calls (the same bits for three cuttings)."""
    cfg = synth.make_small(seed=69, m_ant=4, n_chan=2, s=150000, f_lo=1.2e9, f_s=1e6, n_dm=2, dm_max=50.0,
                           dump_len=1000, ci8=True, n_pulses=2)
    cfg["dm_lists"] = [np.linspace(0.0, 2000.0, 64), np.linspace(0.0, 600.0, 48)]
    ref, lay = run_gpu(cfg, in_dtype="ci8")
    say("classes", lay["n_classes"], "lengths", sorted(set(lay["dm_fft_len"].tolist())))
    assert lay["n_classes"] >= 3
    off = lay["dm_offset"]
    for c in range(2):
        dms = cfg["dm_lists"][c]
        n = lay["dm_fft_len"][off[c]:off[c + 1]]
        v = lay["dm_valid"][off[c]:off[c + 1]]
        l = lay["dm_lead"][off[c]:off[c + 1]]
        keys = set(zip(n.tolist(), v.tolist(), l.tolist()))
        groups = sorted(([d for d in range(len(dms)) if (n[d], v[d], l[d]) == key] for key in keys),
                        key=lambda m: min(dms[d] for d in m))
        top = -1.0
        for members in groups:
            key = (n[members[0]], v[members[0]], l[members[0]])
            dmax = max(dms[d] for d in members)
            assert min(dms[d] for d in members) > top  # classes are contiguous in DM
            top = dmax
            r = oracle.blocking(cfg["chan_freqs"][c], 1e6, dmax, 1000, fft_len=key[0])
            assert (r["fft_len"], r["valid"], r["lead"]) == key
        # the channel's own blocking is that of its largest DM's class (scale window)
        d_top = int(np.argmax(dms))
        assert (lay["fft_len"][c], lay["valid"][c], lay["lead"][c]) == (n[d_top], v[d_top], l[d_top])
    pairs = [(0, 0), (0, 10), (0, 40), (0, 63), (1, 5), (1, 47)]
    err = compare_with_oracle(cfg, ref, lay, pairs=pairs)
    say("classes max normalised error %.3e" % err)
    assert err <= TOL
    for chunks in ([40000, 40000, 70000], [9999, 1, 100000, 40000]):
        got, _ = run_gpu(cfg, in_dtype="ci8", chunks=chunks, max_block=max(chunks))
        assert np.array_equal(got, ref), chunks
    # a spectrum buffer of one class: every class in its own batch, the same bits
    got, lb = run_gpu(cfg, in_dtype="ci8", spectrum_bytes=1)
    assert lb["device_bytes"] < lay["device_bytes"]
    assert np.array_equal(got, ref)


def test_dm_classes_on_the_two_pass_channel(gpu):
    """256 antennas at 0.7 GHz, 16 DMs up to 60 then 32 up to 2990: the low DMs run a
    single-pass class, the others two-pass ones; sampled pairs of each against the oracle."""
    p3 = synth.c3_params()
    cfg = synth.make_small(seed=70, m_ant=256, n_chan=1, s=200000, f_lo=p3["f_lo"], f_s=1e6, n_dm=2,
                           dm_max=3000.0, dump_len=1000, ci8=True, n_pulses=1, radius_m=2500.0)
    cfg["dm_lists"] = [np.concatenate([np.linspace(0.0, 60.0, 16), np.linspace(100.0, 2990.0, 32)])]
    vis, lay = run_gpu(cfg, in_dtype="ci8")
    lens = lay["dm_fft_len"]
    say("classes", lay["n_classes"], "lengths", sorted(set(lens.tolist())))
    assert lay["n_classes"] >= 2 and lens.min() <= 1 << 15 and lens.max() > 1 << 15
    err = compare_with_oracle(cfg, vis, lay, pairs=[(0, 0), (0, 15), (0, 47)])
    say("two-pass classes max normalised error %.3e" % err)
    assert err <= TOL


def test_dm_classes_with_masks_and_compact_records(gpu):
    """Several blocking classes per channel with sparse active DMs (whole classes
    inactive included, which then run no transform): active DMs are bitwise those of
    the full sweep, inactive ones are zeros in full records, and compact records
    hold the same bits for the active pairs."""
    cfg = synth.make_small(seed=71, m_ant=4, n_chan=2, s=120000, f_lo=1.2e9, f_s=1e6, n_dm=2, dm_max=50.0,
                           dump_len=1000, ci8=True, n_pulses=1)
    cfg["dm_lists"] = [np.linspace(0.0, 2000.0, 64), np.linspace(0.0, 600.0, 48)]
    ref, lay = run_gpu(cfg, in_dtype="ci8")
    assert lay["n_classes"] >= 4
    off = lay["dm_offset"]
    # channel 0: a few DMs, none in the top class; channel 1: every fifth DM
    m0 = np.zeros(64, np.uint8)
    m0[[0, 3, 17, 30]] = 1
    m1 = np.zeros(48, np.uint8)
    m1[::5] = 1
    keys = list(zip(lay["dm_fft_len"][off[0]:off[1]].tolist(), lay["dm_valid"][off[0]:off[1]].tolist()))
    assert len({keys[d] for d in np.nonzero(m0)[0]}) < len(set(keys))  # some class wholly inactive
    masked, lm = run_gpu(cfg, in_dtype="ci8", mask=[m0, m1])
    for c, m in enumerate([m0, m1]):
        for d in range(len(m)):
            got = select(masked, lm, c, d)
            if m[d]:
                assert np.array_equal(got, select(ref, lay, c, d)), (c, d)
            else:
                assert not np.any(got), (c, d)
    n_act = int(m0.sum() + m1.sum())
    comp, lc = run_gpu(cfg, in_dtype="ci8", mask=[m0, m1], compact_records=True, max_record_pairs=n_act)
    assert lc["record_pairs"] == n_act
    for c, m in enumerate([m0, m1]):
        for d in np.nonzero(m)[0]:
            assert np.array_equal(select(comp, lc, c, int(d)), select(ref, lay, c, int(d)))


def test_two_pass_forward_beyond_one_grid(gpu):
    """256 antennas, 65536-point (two-pass) transforms, one call of 2^24 samples: the
    forward pre-pass of the call's ~265 blocks needs more (block, antenna) grid rows
    than one launch takes (65535) and runs in slices; the visibilities are bitwise
    those of the same stream in four calls (no slicing)."""
    import torch

    from paper_1109_3186_amd import Plan
    M, N, L, S = 256, 1 << 16, 16000, 1 << 24
    fc = np.array([7.0e8])
    dms = np.array([0.0, 40.0])
    gen = torch.Generator(device=gpu)
    gen.manual_seed(72)
    x = torch.randint(-40, 41, (1, M, 2 * S), generator=gen, dtype=torch.int8, device=gpu)

    def run(chunk, spectrum_bytes):
        outs = []
        with Plan(M, fc, 1e6, L, max_block_samples=chunk, in_dtype="ci8", fft_len=N,
                  spectrum_bytes=spectrum_bytes) as p:
            p.set_dm_trials(dms)
            lay = p.layout()
            for s0 in range(0, S, chunk):
                p.process_block(x[..., 2 * s0:2 * (s0 + chunk)].contiguous(), flush=(s0 + chunk >= S))
                _, nd, vis = p.fetch()
                if nd:
                    outs.append(vis.clone())
            torch.cuda.synchronize()
        return torch.cat(outs), lay

    one, lay = run(S, 48 << 30)
    blocks = -(-S // int(lay["valid"][0]))
    say("one call: V %d, ~%d blocks x %d antennas = %d pre-pass rows" % (lay["valid"][0], blocks, M, blocks * M))
    assert int(lay["fft_len"][0]) == N and blocks * M > 65535
    four, _ = run(S // 4, 0)
    assert one.shape == four.shape and one.shape[0] == S // L
    assert torch.equal(one, four)
    del one, four, x
    torch.cuda.empty_cache()
