"""The 36-antenna workload at full size, in the launch configuration bench.py times
(64 channels x 2^20 complex-int8 samples, 256 DMs over 0-2000, 1 ms dumps,
stream fed in 2^18-sample calls): sampled (channel, DM) outputs against the FP64
oracle, and recovery of every injected pulse at its DM."""
import numpy as np
import pytest

import oracle
import synth
from gpu_helpers import blockings, norm_error, say

pytestmark = pytest.mark.gpu

PAIRS = [(0, 255), (31, 128), (63, 0), (63, 201)]
CHUNK = 1 << 18


@pytest.fixture(scope="module")
def c1_input(gpu):
    import torch
    p = synth.c1_params()
    say("building the 36-antenna stream on the device")
    x, pulses, fc, pos = synth.make_stream_device(p, gpu)
    chunks = [x[..., 2 * s0:2 * min(p["samples"], s0 + CHUNK)].contiguous() for s0 in range(0, p["samples"], CHUNK)]
    host = {c: np.concatenate([ch[c].cpu().numpy() for ch in chunks], axis=-1) for c in sorted({c for c, _ in PAIRS})}
    del x
    torch.cuda.synchronize()
    return p, chunks, pulses, fc, host


def _run(p, chunks, fc, corr, pairs=None, extra=None):
    import torch

    import bench
    from paper_1109_3186_amd import Plan
    dms = synth.dm_grid(p["n_dm"], p["dm_max"])
    # the schedule bench.py runs (the tuned entry of the FP32 workload for every form)
    kw, schedule = bench.c1_schedule(p, fc, dms, "f32", CHUNK)
    kw.update(extra or {})
    say("schedule: %s %s" % (schedule, extra or ""))
    plan = Plan(p["m_ant"], fc, p["f_s"], p["dump_len"], max_block_samples=CHUNK, in_dtype="ci8", corr_dtype=corr,
                **kw)
    plan.set_dm_trials(dms)
    lay = plan.layout()
    m = p["m_ant"]
    nbl = lay["n_baselines"]
    iu, ju = np.triu_indices(m)
    auto_idx = torch.tensor(np.nonzero(iu == ju)[0], device="cuda")
    pairs = PAIRS if pairs is None else pairs
    keep = {pair: [] for pair in pairs}
    power = []
    for i, ch in enumerate(chunks):
        plan.process_block(ch, flush=(i == len(chunks) - 1))
        _, nd, vis = plan.fetch()
        if not nd:
            continue
        v = vis.view(nd, -1, nbl)  # [dump, (c, d), baseline]
        power.append(v.index_select(2, auto_idx).real.sum(dim=2).cpu().numpy())
        for (c, d) in pairs:
            keep[(c, d)].append(v[:, lay["dm_offset"][c] + d].cpu().numpy())
        del vis, v
        torch.cuda.synchronize()
    lay = plan.layout()
    plan.close()
    return {k: np.concatenate(v) for k, v in keep.items()}, np.concatenate(power), lay, dms


def test_c1_sampled_parity_and_pulses(c1_input):
    p, chunks, pulses, fc, host = c1_input
    say("F32 run")
    got, power, lay, dms = _run(p, chunks, fc, "f32")
    assert power.shape[0] == p["samples"] // p["dump_len"]
    bl = blockings(lay)
    worst = 0.0
    for (c, d), v in got.items():
        say("oracle for channel %d DM trial %d" % (c, d))
        ref = oracle.run_oracle(host[c][None], fc[c:c + 1], p["f_s"], [dms], p["dump_len"], [bl[c]], chans=[0],
                                dm_index=[d])[(0, d)]
        e = norm_error(v, ref, p["m_ant"])
        say("  max normalised error %.3e" % e)
        worst = max(worst, e)
    assert worst <= 1e-5
    # every injected pulse is recovered within one trial of its DM: sum each
    # channel's auto power at the dump where trial d puts the pulse (the exported
    # channel shifts, relative to the highest channel centre, carry the DM delay)
    pw = power.reshape(power.shape[0], p["n_chan"], p["n_dm"])
    shift = lay["shift"].reshape(p["n_chan"], p["n_dm"])
    for pl in pulses:
        score = np.zeros(p["n_dm"])
        for d in range(p["n_dm"]):
            m = (pl["n0"] + pl["width"] // 2 + shift[:, d]) // p["dump_len"]
            ok = m < pw.shape[0]
            score[d] = pw[m[ok], np.nonzero(ok)[0], d].sum()
        best = int(np.argmax(score))
        true = pl["dm"] / (p["dm_max"] / p["n_dm"])
        say("pulse DM %.1f (trial %.2f) -> best trial %d" % (pl["dm"], true, best))
        assert abs(best - true) <= 1.0 + 1e-9


# Reduced-precision inputs round only the products between antennas; the
# autocorrelations are the dumps' power of the unrounded voltages.  The bound is on
# the maximum over every sampled visibility, the DM 0 trial included.
@pytest.mark.parametrize("corr,bound", [("e4m3", 1e-2), ("f16", 1e-4)])
def test_c1_quantised_error_table(c1_input, corr, bound):
    p, chunks, pulses, fc, host = c1_input
    say("%s run" % corr)
    got, power, lay, dms = _run(p, chunks, fc, corr)
    bl = blockings(lay)
    iu, ju = np.triu_indices(p["m_ant"])
    allerr, dm0 = [], [np.zeros(0)]
    for (c, d), v in got.items():
        ref = oracle.run_oracle(host[c][None], fc[c:c + 1], p["f_s"], [dms], p["dump_len"], [bl[c]], chans=[0],
                                dm_index=[d])[(0, d)]
        auto = ref[:, iu == ju].real
        norm = np.sqrt(auto[:, iu] * auto[:, ju])
        err = (np.abs(v.astype(np.complex128) - ref) / norm).ravel()
        (dm0 if d == 0 else allerr).append(err)
    e = np.concatenate(allerr)
    z = np.concatenate(dm0)
    say("%s vs FP64 oracle over %d visibilities (DM > 0): max %.3e, 99.9%% %.3e, rms %.3e; DM 0: max %.3e; "
        "scales %s" % (corr, e.size, e.max(), np.quantile(e, 0.999), np.sqrt(np.mean(e ** 2)), z.max(),
                       np.unique(lay["scale"])))
    assert e.max() <= bound
    assert z.max() <= bound


def test_c1_learned_proposal(c1_input):
    """The learned proposal on the full-size stream, in the plan configuration bench.py
    times for it (the tuned schedule, one blocking class per channel): every injected
    pulse's DM trial is kept (or the proposal falls back to the full sweep), and
    visibilities of the kept DMs are bitwise those of the full sweep with the same
    options."""
    import math
    import os

    import torch

    import bench
    from paper_1109_3186_amd import Plan
    from paper_1109_3186_amd.proposal import Proposal, load_weights
    p, chunks, pulses, fc, host = c1_input
    wpath = os.path.join(os.path.dirname(os.path.dirname(__file__)), "paper_1109_3186_amd", "proposal_weights.npz")
    dms = synth.dm_grid(p["n_dm"], p["dm_max"])
    kw, _ = bench.c1_schedule(p, fc, dms, "f32", CHUNK)
    plan = Plan(p["m_ant"], fc, p["f_s"], p["dump_len"], max_block_samples=CHUNK, in_dtype="ci8",
                dm_classes="single", **kw)
    plan.set_dm_trials(dms)
    full = torch.cat(chunks, dim=-1).contiguous()
    prop = Proposal(plan, load_weights(wpath), budget=0.1)
    mask, scores, fb = prop.select(full)
    del full
    dstep = p["dm_max"] / p["n_dm"]
    hits = [bool(mask[math.floor(q["dm"] / dstep)] or mask[min(math.ceil(q["dm"] / dstep), p["n_dm"] - 1)])
            for q in pulses]
    say("learned proposal: %d active, fallback %s, recall %d/%d" % (mask.sum(), fb, sum(hits), len(hits)))
    assert all(hits)
    plan.set_active_dms(mask)
    lay = plan.layout()
    nbl = lay["n_baselines"]
    active = np.nonzero(mask)[0][:3]
    got = {d: [] for d in active}
    for i, ch in enumerate(chunks):
        plan.process_block(ch, flush=(i == len(chunks) - 1))
        _, nd, vis = plan.fetch()
        v = vis.view(nd, -1, nbl)
        for d in active:
            got[d].append(v[:, lay["dm_offset"][63] + d].cpu().numpy())
    prop.close()
    plan.close()
    ref, _, _, _ = _run(p, chunks, fc, "f32", pairs=[(63, int(d)) for d in active], extra={"dm_classes": "single"})
    for d in active:
        assert np.array_equal(np.concatenate(got[d]), ref[(63, int(d))])
