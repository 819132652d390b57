"""The 256-antenna workload at full size, in the launch configuration bench.py
times (256 antennas, 32 x 1 MHz channels at 0.7-0.732 GHz, 2^18 complex-int8
samples, per-channel DM grids of 512..1536 trials over 0-3000 in blocking classes
of single-pass and two-pass transforms, the stream run once per DM window into
compact records): sampled (channel, DM) outputs of the passes that hold them
against the FP64 oracle."""
import numpy as np
import pytest

import oracle
from gpu_helpers import blockings, norm_error, say

pytestmark = pytest.mark.gpu


def test_c3_full_size_sampled(gpu):
    import torch

    import bench
    say("building the 256-antenna stream and plan (bench configuration)")
    st = bench.c3_setup(gpu, "f32", False, 0)
    p, windows, plan = st["p"], st["windows"], st["plan"]
    n_dm, L = p["n_dm"], p["dump_len"]
    lay0 = plan.layout()
    # the first channel's highest DM (two-pass, the longest transform), a third of the
    # way up the last channel's grid, and DM 0 of a middle channel (its lowest class)
    pairs = [(0, n_dm[0] - 1), (31, n_dm[31] // 3), (13, 0)]
    for c, d in pairs:
        say("pair (%d, %d): DM %.1f, transform %d points" % (
            c, d, st["dms"][c][d], lay0["dm_fft_len"][lay0["dm_offset"][c] + d]))
    lengths = {int(lay0["dm_fft_len"][lay0["dm_offset"][c] + d]) for c, d in pairs}
    assert max(lengths) > 1 << 15 and min(lengths) <= 1 << 15  # two-pass and single-pass classes
    by_pass = {}
    for c, d in pairs:
        k = next(k for k in range(st["passes"]) if d in windows[c][k])
        by_pass.setdefault(k, []).append((c, d))
    got = {}
    for k, kp in sorted(by_pass.items()):
        say("pass %d of %d" % (k, st["passes"]))
        nd = bench.c3_pass(st, k)
        torch.cuda.synchronize()
        lay = plan.layout()
        nbl, rec = lay["n_baselines"], lay["record_elems"]
        assert nd == p["samples"] // L
        vis = st["out"].view(-1)[:nd * rec].view(nd, rec)  # fetch packs [dump][record]
        for c, d in kp:
            o = int(lay["record_pos"][lay["dm_offset"][c] + d])
            assert o >= 0
            got[(c, d)] = vis[:, o * nbl:(o + 1) * nbl].cpu().numpy()
    bl = blockings(plan.layout())
    host = {c: st["x"][c].cpu().numpy() for c in {c for c, _ in pairs}}
    fc, dms = st["fc"], st["dms"]
    plan.close()
    st.clear()
    torch.cuda.empty_cache()
    worst = 0.0
    for (c, d), v in got.items():
        say("oracle for channel %d DM trial %d" % (c, d))
        ref = oracle.run_oracle(host[c][None], fc[c:c + 1], p["f_s"], [dms[c]], L, [bl[c]], chans=[0],
                                dm_index=[d])[(0, d)]
        assert v.shape == ref.shape
        e = norm_error(v, ref, p["m_ant"])
        say("  max normalised error %.3e" % e)
        worst = max(worst, e)
    assert worst <= 1e-5
