"""Autotuner of the plan's tile and schedule parameters, with a JSON cache.

What it chooses, by timing the library on the device (synthetic complex-int8
noise, the workload's own antennas, channels and DM grids):

* the cost model from which a plan cuts each channel's DMs into blocking classes
  and picks every class's transform length (ddx_set_dm_trials): the time per
  transform point of the inverse (chirp multiply, inverse FFT, discard) and of the
  forward transform at every length 2^8 .. 2^18, from the library's own kernel
  timings on a stream of the workload's antennas, call size and correlator format;
* the wave size (units per dedispersion / correlator launch) and the DM group
  (DMs run back to back on one spectrum block), by timing whole streams of up to
  8 of the workload's channels with that cost model in force.

Throughput is measured as antenna-samples x DM trials per second over a whole
short stream (process_block + fetch into device memory), processed in calls of
the workload's own size (max_block).  Results are cached in a JSON file keyed by
the device, the workload and TUNE_VERSION (raised when the search or the kernels'
trade-offs change), so a later run with the same key costs nothing.
"""
import hashlib
import json
import math
import os
import time

import numpy as np

from .binding import DdxError, Plan, plan_blocking

DEFAULT_CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tune_cache.json")
MIN_LOG, MAX_LOG = 8, 18
TUNE_VERSION = 4


def device_id():
    """The device as the cache knows it: architecture and compute-unit count (the
    marketing name the runtime reports depends on an ids file that may be absent)."""
    import torch
    prop = torch.cuda.get_device_properties(0)
    return "%s x %d CU" % (prop.gcnArchName.split(":")[0], prop.multi_processor_count)


def key_of(desc):
    return hashlib.sha256(json.dumps(desc, sort_keys=True).encode()).hexdigest()[:24]


def workload_key(n_ant, chan_freqs, samp_rate, dump_len, dm_lists, corr_dtype, in_dtype, max_block):
    desc = {
        "device": device_id(), "version": TUNE_VERSION, "n_ant": int(n_ant),
        "chan_freqs": [float(f) for f in chan_freqs], "samp_rate": float(samp_rate), "dump_len": int(dump_len),
        "dms": hashlib.sha256(np.concatenate([np.asarray(d, np.float64) for d in dm_lists]).tobytes()).hexdigest()[:16],
        "n_dm": [int(len(d)) for d in dm_lists], "corr": corr_dtype, "in": in_dtype, "max_block": int(max_block),
    }
    return key_of(desc), desc


def _noise(n_chan, n_ant, n, in_dtype, seed):
    import torch
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    if in_dtype == "ci8":
        x = torch.randn((n_chan, n_ant, 2 * n), generator=g, device="cuda") * 16.0
        return x.round_().clamp_(-127, 127).to(torch.int8)
    return torch.randn((n_chan, n_ant, n), generator=g, device="cuda", dtype=torch.complex64)


def _time_stream(plan, x, repeats=2):
    """Best wall time of one whole stream (process_block in max-size chunks + fetch)."""
    import torch
    lay = plan.layout()
    mb = plan.max_block
    n = x.shape[-1] // 2 if plan.in_dtype == "ci8" else x.shape[-1]
    per = 2 if plan.in_dtype == "ci8" else 1
    chunks = [x[..., per * s0:per * min(n, s0 + mb)].contiguous() for s0 in range(0, n, mb)]
    out = torch.empty((lay["ring_dumps"], max(lay["record_elems"], 1)), dtype=torch.complex64, device="cuda")
    best = float("inf")
    for _ in range(repeats + 1):  # first run warms up
        plan.reset_stream()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i, c in enumerate(chunks):
            plan.process_block(c, flush=(i == len(chunks) - 1))
            plan.fetch(out=out)
        torch.cuda.synchronize()
        best = min(best, time.perf_counter() - t0)
    return best


def _sample_dms(dms, k):
    """k trials of a DM list, always including the largest."""
    dms = np.asarray(dms, np.float64)
    if len(dms) <= k:
        return dms
    idx = np.unique(np.concatenate([np.linspace(0, len(dms) - 1, k).round().astype(int), [int(np.argmax(dms))]]))
    return dms[idx]


def measure_costs(n_ant, chan_freq, samp_rate, dump_len, corr_dtype="f32", in_dtype="ci8", max_block=1 << 18,
                  n_dm=16, log=None):
    """Picoseconds per transform point of the inverse and forward transforms at N =
    2^8 .. 2^18, as [[inverse x 11], [forward x 11]], from the library's kernel
    timings (ddx_set_profiling) on one channel: n_dm trials at DM 0 (a transform's
    cost does not depend on the chirp's values), a stream of at least four blocks in
    calls of max_block.  A length too short to keep one dump takes the value of the
    next measured length (no plan can choose it)."""
    import torch
    say = log or (lambda *a: None)
    inv, fwd = {}, {}
    for l in range(MIN_LOG, MAX_LOG + 1):
        n = 1 << l
        if n < dump_len:
            continue
        s = max(4 * n, min(max_block, 1 << 18))
        mb = min(max_block, s)
        x = _noise(1, n_ant, s, in_dtype, seed=1112)
        try:
            with Plan(n_ant, [chan_freq], samp_rate, dump_len, max_block_samples=mb, in_dtype=in_dtype,
                      corr_dtype=corr_dtype, fft_len=n, ring_dumps=s // dump_len + 4) as p:
                p.set_dm_trials(np.zeros(n_dm))
                _time_stream(p, x, repeats=0)  # warm-up
                p.set_profiling(True)
                _time_stream(p, x, repeats=0)
                pr = p.profile()
        except DdxError as e:
            say("length %d: %s" % (n, e))
            continue
        finally:
            del x
        d, f = pr["dedisperse"], pr["forward"]
        inv[l] = d["time_ms"] * 1e9 / (d["flops"] / (5 * l + 6))
        fwd[l] = f["time_ms"] * 1e9 / (f["flops"] / (5 * l))
        say("length %d: inverse %.3f ps, forward %.3f ps per point" % (n, inv[l], fwd[l]))
        torch.cuda.synchronize()
    if not inv:
        raise RuntimeError("no transform length could be measured")
    table = [[0.0] * (MAX_LOG - MIN_LOG + 1) for _ in range(2)]
    for l in range(MAX_LOG, MIN_LOG - 1, -1):
        nxt = min((k for k in inv if k >= l), default=max(inv))
        table[0][l - MIN_LOG] = inv.get(l, inv[nxt])
        table[1][l - MIN_LOG] = fwd.get(l, fwd[nxt])
    return table


def cached(n_ant, chan_freqs, samp_rate, dump_len, dm_lists, corr_dtype="f32", in_dtype="ci8", max_block=1 << 18,
           cache=DEFAULT_CACHE):
    """The cached tune() result for the workload on this device, or None (measures nothing)."""
    key, _ = workload_key(n_ant, chan_freqs, samp_rate, dump_len, dm_lists, corr_dtype, in_dtype, max_block)
    if not cache or not os.path.exists(cache):
        return None
    with open(cache) as f:
        db = json.load(f)
    if key not in db:
        return None
    r = dict(db[key])
    r["source"] = "cache"
    return r


def tune(n_ant, chan_freqs, samp_rate, dump_len, dm_lists, corr_dtype="f32", in_dtype="ci8", max_block=1 << 18,
         cache=DEFAULT_CACHE, force=False, dm_sample=16, log=None):
    """Return {"cost_ps": [[...], [...]], "wave_units": W, "dm_group": G, ...} for the
    workload, from the cache when present, else by measurement (then cached)."""
    say = log or (lambda *a: None)
    key, desc = workload_key(n_ant, chan_freqs, samp_rate, dump_len, dm_lists, corr_dtype, in_dtype, max_block)
    db = {}
    if cache and os.path.exists(cache):
        with open(cache) as f:
            db = json.load(f)
    if not force and key in db:
        r = dict(db[key])
        r["source"] = "cache"
        return r
    t_start = time.time()
    chan_freqs = np.asarray(chan_freqs, np.float64)
    n_chan = len(chan_freqs)
    # 1. the classes' cost model, on the channel of the longest smear
    rep = int(np.argmin(chan_freqs))
    cost = measure_costs(n_ant, float(chan_freqs[rep]), samp_rate, dump_len, corr_dtype, in_dtype, max_block,
                         log=say)
    # 2. wave size and DM group on up to 8 channels with sampled DMs, as many
    # (channel, DM) pairs as keep the stream's visibilities within a few GB
    sub = list(range(0, n_chan, max(1, n_chan // 8)))[:8]
    s = min(max_block, 1 << 18)
    nbl = n_ant * (n_ant + 1) // 2
    ring = s // dump_len + 2
    pairs = max(2 * len(sub), int(8e9 // (ring * nbl * 8)))
    per_chan = max(2, min(4 * dm_sample, pairs // len(sub)))
    dm_sub = [_sample_dms(dm_lists[c], per_chan) for c in sub]
    x = _noise(len(sub), n_ant, s, in_dtype, seed=1114)
    # bytes one unit occupies in a wave: its voltages (and two-pass rows)
    y_bytes = {"f32": 8, "f16": 4, "e4m3": 2}[corr_dtype]
    per_unit = 0
    for i, c in enumerate(sub):
        n, v, _, _ = plan_blocking([chan_freqs[c]], samp_rate, dump_len, dm_sub[i], cost_ps=cost)
        per_unit = max(per_unit, n_ant * int(v.max()) * y_bytes + (n_ant * int(n.max()) * 8 if n.max() > 1 << 15 else 0))
    sched = {}
    for wu in (0, 16, 64, 128, 256, 512):
        if wu and wu * per_unit > 16e9:
            continue
        for dg in (8, 16, 32):
            try:
                with Plan(n_ant, chan_freqs[sub], samp_rate, dump_len, max_block_samples=s, in_dtype=in_dtype,
                          corr_dtype=corr_dtype, cost_ps=cost, wave_units=wu, dm_group=dg, ring_dumps=ring) as p:
                    for i, d in enumerate(dm_sub):
                        p.set_dm_trials(d, chan=i)
                    t = _time_stream(p, x)
                    units = n_ant * s * sum(len(d) for d in dm_sub)
                    sched["%d/%d" % (wu, dg)] = units / t
                    say("wave %d, DM group %d: %.3e units/s" % (wu, dg, units / t))
            except DdxError as e:
                say("wave %d, DM group %d: %s" % (wu, dg, e))
    del x
    best = max(sched, key=sched.get)
    wu, dg = (int(v) for v in best.split("/"))
    r = {"cost_ps": cost, "wave_units": wu, "dm_group": dg, "schedule_trials": sched,
         "seconds": round(time.time() - t_start, 1), "workload": desc}
    if cache:
        db[key] = r
        tmp = cache + ".tmp"
        with open(tmp, "w") as f:
            json.dump(db, f, indent=1, sort_keys=True)
        os.replace(tmp, cache)
    r = dict(r)
    r["source"] = "measured"
    return r


def plan_kwargs(tuned):
    """Plan keyword arguments from a tune() result."""
    return {"cost_ps": tuned["cost_ps"], "wave_units": tuned["wave_units"], "dm_group": tuned["dm_group"]}


if __name__ == "__main__":
    import argparse
    import sys
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    import synth
    ap = argparse.ArgumentParser(description="tune a named workload and cache the result")
    ap.add_argument("workload", choices=["c1", "c3"])
    ap.add_argument("--corr", default="f32", choices=["f32", "f16", "e4m3"])
    ap.add_argument("--force", action="store_true")
    ap.add_argument("--cache", default=DEFAULT_CACHE, help="JSON cache file")
    a = ap.parse_args()
    p = synth.c1_params() if a.workload == "c1" else synth.c3_params()
    fc = synth.chan_freqs(p["f_lo"], p["n_chan"], p["f_s"])
    nd = p["n_dm"] if isinstance(p["n_dm"], list) else [p["n_dm"]] * p["n_chan"]
    dms = [synth.dm_grid(n, p["dm_max"]) for n in nd]
    res = tune(p["m_ant"], fc, p["f_s"], p["dump_len"], dms, corr_dtype=a.corr,
               max_block=(1 << 18) if a.workload == "c1" else p["samples"], cache=a.cache, force=a.force,
               log=lambda *m: print(*m, flush=True))
    print(json.dumps({k: res[k] for k in ("cost_ps", "wave_units", "dm_group", "source")}))
