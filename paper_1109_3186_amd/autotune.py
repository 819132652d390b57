"""Autotuner of the plan's tile and schedule parameters, with a JSON cache.

What it chooses, by timing the library on the device (synthetic complex-int8
noise, the workload's own channels and DM grids):

* the transform length N_c of each channel: the automatic length (the smallest
  power of two keeping at least half of each block), half of it when that still
  keeps a whole dump, and two and four times it up to 2^18.  A longer transform
  keeps more of each block (V_c / N_c grows) at a higher cost per point; above
  2^15 it also takes the two-pass path.  Channels whose automatic length agrees
  are tuned together on the one with the longest dispersion smear;
* the wave size (units per dedispersion / correlator launch) and the DM group
  (DMs run back to back on one spectrum block).

Throughput is measured as antenna-samples x DM trials per second over a whole
short stream (process_block + fetch into device memory), processed in calls of
the workload's own size (max_block), so that the block count of each length is
the one the workload will see.  Results are cached in a JSON file keyed by the
device, the workload and TUNE_VERSION (raised when the search or the kernels'
trade-offs change), so a later run with the same key costs nothing.
"""
import hashlib
import json
import math
import os
import time

import numpy as np

from .binding import DdxError, Plan

DEFAULT_CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tune_cache.json")
MAX_LEN = 1 << 18
TUNE_VERSION = 3


def workload_key(n_ant, chan_freqs, samp_rate, dump_len, dm_lists, corr_dtype, in_dtype, max_block):
    import torch
    desc = {
        "device": torch.cuda.get_device_name(0), "version": TUNE_VERSION, "n_ant": int(n_ant),
        "chan_freqs": [float(f) for f in chan_freqs], "samp_rate": float(samp_rate), "dump_len": int(dump_len),
        "dms": hashlib.sha256(np.concatenate([np.asarray(d, np.float64) for d in dm_lists]).tobytes()).hexdigest()[:16],
        "n_dm": [int(len(d)) for d in dm_lists], "corr": corr_dtype, "in": in_dtype, "max_block": int(max_block),
    }
    return hashlib.sha256(json.dumps(desc, sort_keys=True).encode()).hexdigest()[:24], desc


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
    """k trials of a DM list, always including the largest (it fixes the blocking)."""
    dms = np.asarray(dms, np.float64)
    if len(dms) <= k:
        return dms
    idx = np.unique(np.concatenate([np.linspace(0, len(dms) - 1, k).round().astype(int), [int(np.argmax(dms))]]))
    return dms[idx]


def _auto_lengths(n_ant, chan_freqs, samp_rate, dump_len, dm_lists, in_dtype):
    with Plan(n_ant, chan_freqs, samp_rate, dump_len, max_block_samples=1 << 16, in_dtype=in_dtype) as p:
        for c, d in enumerate(dm_lists):
            p.set_dm_trials(_sample_dms(d, 1), chan=c)
        lay = p.layout()
        return [int(n) for n in lay["fft_len"]], [int(v) for v in lay["valid"]]


def tune(n_ant, chan_freqs, samp_rate, dump_len, dm_lists, corr_dtype="f32", in_dtype="ci8", max_block=1 << 18,
         cache=DEFAULT_CACHE, force=False, dm_sample=16, log=None):
    """Return {"fft_len": [...], "wave_units": W, "dm_group": G, ...} for the workload,
    from the cache when present, else by measurement (then cached)."""
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
    auto_n, auto_v = _auto_lengths(n_ant, chan_freqs, samp_rate, dump_len, dm_lists, in_dtype)
    # 1. transform length per group of channels sharing the automatic length
    chosen = list(auto_n)
    length_trials = {}
    for n0 in sorted(set(auto_n)):
        members = [c for c in range(n_chan) if auto_n[c] == n0]
        rep = min(members, key=lambda c: auto_v[c])  # longest smear of the group
        dms = _sample_dms(dm_lists[rep], dm_sample)
        cands = [n for n in (n0 // 2, n0, 2 * n0, 4 * n0) if 256 <= n <= MAX_LEN]
        # the workload's call size when it holds a block of every candidate, else four blocks
        s = max_block if max_block >= max(cands) else max(4 * max(cands), 1 << 17)
        x = _noise(1, n_ant, s, in_dtype, seed=1113)
        rates = {}
        for n in cands:
            try:
                with Plan(n_ant, chan_freqs[rep:rep + 1], samp_rate, dump_len, max_block_samples=s,
                          in_dtype=in_dtype, corr_dtype=corr_dtype, fft_len=n, ring_dumps=s // dump_len + 4) as p:
                    p.set_dm_trials(dms)
                    t = _time_stream(p, x)
                    rates[n] = n_ant * s * len(dms) / t
                    say("length %d (channel %d): %.3e units/s" % (n, rep, rates[n]))
            except DdxError as e:  # too short for the smear, or out of memory
                say("length %d (channel %d): %s" % (n, rep, e))
        del x
        best = max(rates, key=rates.get)
        length_trials[str(n0)] = {str(k): v for k, v in rates.items()}
        for c in members:
            chosen[c] = best
    # 2. wave size and DM group on up to 8 channels with sampled DMs, as many
    # (channel, DM) pairs as keep the stream's visibilities within a few GB
    sub = list(range(0, n_chan, max(1, n_chan // 8)))[:8]
    s = max(2 * max(chosen[c] for c in sub), min(max_block, 1 << 18))
    nbl = n_ant * (n_ant + 1) // 2
    ring = s // dump_len + 2
    pairs = max(2 * len(sub), int(8e9 // (ring * nbl * 8)))
    per_chan = max(2, min(4 * dm_sample, pairs // len(sub)))
    dm_sub = [_sample_dms(dm_lists[c], per_chan) for c in sub]
    x = _noise(len(sub), n_ant, s, in_dtype, seed=1114)
    y_bytes = {"f32": 8, "f16": 4, "e4m3": 2}[corr_dtype]
    # bytes one unit occupies in a wave (V_c < N_c bounds the dedispersed row)
    per_unit = n_ant * max(chosen) * y_bytes + (n_ant * max(chosen) * 8 if max(chosen) > (1 << 15) else 0)
    sched = {}
    for wu in (0, 16, 64, 128, 256, 512):
        if wu and wu * per_unit > 16e9:
            continue
        for dg in (8, 16, 32):
            try:
                with Plan(n_ant, chan_freqs[sub], samp_rate, dump_len, max_block_samples=s,
                          in_dtype=in_dtype, corr_dtype=corr_dtype, fft_len=[chosen[c] for c in sub],
                          wave_units=wu, dm_group=dg, ring_dumps=ring) as p:
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
    r = {"fft_len": chosen, "wave_units": wu, "dm_group": dg, "auto_fft_len": auto_n,
         "length_trials": length_trials, "schedule_trials": sched, "seconds": round(time.time() - t_start, 1),
         "workload": desc}
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
    return {"fft_len": tuned["fft_len"], "wave_units": tuned["wave_units"], "dm_group": tuned["dm_group"]}


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
    print(json.dumps({k: res[k] for k in ("fft_len", "wave_units", "dm_group", "source")}))
