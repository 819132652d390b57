#!/usr/bin/env python3
"""Throughput of the coherent-dedispersion correlator on one MI355X.

One step = the whole pre-integrator stage over one synthetic stream of the
36-antenna workload (64 x 1 MHz channels at 1.2-1.264 GHz, 2^20 complex-int8
samples per channel and antenna, 256 trial DMs over 0-2000 pc cm^-3, 1 ms
dumps, 10 injected pulses): overlap-save forward FFT, chirp generation, chirp
multiply + inverse FFT for every DM, cross-multiply and integrate-and-dump of
all 666 baselines, and the fetch of every dump record into device memory.
The input is resident in HBM before the timed region.

Prints one JSON line.  --gpus above 1 is refused: the library has no multi-GPU path.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "antenna-samples×DM-trials/s correlated; % HBM/MFMA peak; learned vs plain speedup"
UNIT = "antenna-samples*DM-trials/s"
PEAKS = {  # MI355X published dense peaks
    "hbm_gbs": 8000.0, "fp32_vector_tflops": 157.3, "fp32_mfma_tflops": 157.3, "fp16_mfma_tflops": 2500.0,
    "fp8_mfma_tflops": 5000.0,
    # FP32 FMA without packed instructions: 256 CU x 4 SIMD x 16 lanes x 2 flop x 2.4 GHz
    # (the published vector figure counts two FMAs per lane per cycle, from packed FP32)
    "fp32_vector_unpacked_tflops": 256 * 4 * 16 * 2 * 2.4e9 / 1e12,
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# the translation unit that holds k_dedisperse and k_correlate (the network's
# kernels are compiled from cnn.hip alone)
DEDISP_SOURCES = ("fft.hpp", "kernels.hpp", "ddx.hip", "tiles.hpp")
IMAGE_SOURCES = ("image.hip",)
INCOHERENT_SOURCES = ("incoherent.hip",)
CHIMG_SOURCES = ("chimg.hip",)


# The paper reports no measured numbers: its figures are analytic operation rates,
# counted as one complex multiply-accumulate per op, for an SKA-like workload
# (400 MHz, 12 m dishes, 1 km longest baseline, 1.4 GHz, 2 polarisations, DMs 10-1000
# in a geometric bank of ratio 1.1).  Evaluated here at M = 36 antennas: the
# Chirpolator's DFT step (Sec. 5.1, App. A.4, with the factorisation's rho_f = 0.61,
# only the bins a baseline needs); coherent dedispersion over many DMs it only calls
# prohibitive (Sec. 2.3.2).  Context for the units/s above, not a target.
PAPER_CONTEXT = {
    "chirpolator_dft_complex_op_per_s_36_antennas": 4.3e14,
    "assumptions": "SKA-like: 400 MHz, 12 m dishes, 1 km max baseline, 1.4 GHz, 2 pol, DM 10-1000 (48 trials), "
                   "1 complex MAC = 1 op, rho_f = 0.61, only the needed bins",
    "coherent_dedispersion": "no op count: called prohibitive for many DMs",
}


def kernel_source_hash(sources=DEDISP_SOURCES):
    h = hashlib.sha256()
    for f in sources:
        with open(os.path.join(ROOT, "paper_1109_3186_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel, workload, sources=DEDISP_SOURCES):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it
    was taken on the current kernel sources; else None."""
    path = os.path.join(ROOT, "profiles", "traffic_%s_%s.json" % (kernel, workload))
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    if t.get("source_hash") != kernel_source_hash(sources):
        return None
    return t.get("bytes_per_launch")


def blocking_desc(lay):
    """The plan's overlap-save blocking in a few words: the transform lengths in use
    and the DM classes (each channel's DMs cut into classes with their own length)."""
    lens = "/".join(str(n) for n in sorted(set(int(v) for v in lay["dm_fft_len"])))
    return "N %s in %d DM classes over %d channels" % (lens, lay["n_classes"], lay["n_chan"])


def build_input(p, dev, chunk):
    import torch

    import synth
    t0 = time.time()
    x, pulses, fc, pos = synth.make_stream_device(p, dev)
    s = p["samples"]
    chunks = []
    for s0 in range(0, s, chunk):
        s1 = min(s, s0 + chunk)
        chunks.append(x[..., 2 * s0:2 * s1].contiguous())
    del x
    torch.cuda.synchronize()
    torch.cuda.empty_cache()  # the generator's temporaries go back to the device for the plans
    log("input built in %.1f s: %d chunks" % (time.time() - t0, len(chunks)))
    return chunks, pulses, fc


def host_cpu():
    """Host threads available to this process (at most 16, the CPU share of one GPU)
    and the CPU model."""
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 1
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.startswith("model name"):
                    model = ln.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return min(16, avail), avail, model


def cpu_baseline(chunks, fc, dms, lay, p, per_thread):
    """The FP64 oracle on all host threads: channel 0, `per_thread` DM trials per
    thread spread over the grid, all antennas, the whole time span; units/s scaled to
    the metric's unit.  numpy's FFTs and matrix products release the GIL, so one
    Python thread per DM trial runs in parallel (each with single-threaded BLAS)."""
    from concurrent.futures import ThreadPoolExecutor

    import numpy as np
    from threadpoolctl import threadpool_limits

    import oracle
    threads, avail, model = host_cpu()
    x = np.concatenate([c[0].cpu().numpy() for c in chunks], axis=-1)[None]
    from paper_1109_3186_amd import layout_blockings
    bl = layout_blockings(lay)[:1]
    n_dm = min(len(dms), threads * per_thread)
    ds = [int(v) for v in np.linspace(0, len(dms) - 1, n_dm).round()]
    parts = [ds[i::threads] for i in range(threads)]

    def work(part):
        return oracle.run_oracle(x, fc[:1], p["f_s"], [dms], p["dump_len"], bl, chans=[0], dm_index=part)

    with threadpool_limits(limits=1):
        t0 = time.time()
        with ThreadPoolExecutor(threads) as ex:
            outs = [o for o in ex.map(work, [q for q in parts if q])]
        el = time.time() - t0
    nd = next(iter(outs[0].values())).shape[0]
    units = p["m_ant"] * nd * p["dump_len"] * len(ds)
    return {"value": units / el, "unit": UNIT, "cores": threads, "kind": "oracle",
            "sample": "channel 0 x %d DMs spread over the grid x %d antennas x %d samples, FP64 numpy, one DM "
                      "per thread at a time on %d threads, %.1f s" % (len(ds), p["m_ant"], p["samples"], threads, el),
            "host": {"nproc": avail, "threads_used": threads, "cpu_model": model}}


def weights_provenance(path):
    """How the committed proposal weights were trained (from the file's metadata)."""
    import json

    import numpy as np
    with np.load(path) as z:
        meta = json.loads(str(z["meta"])) if "meta" in z else {}
    return "trained in %s on %s tiles" % (meta.get("precision", "fp32"), meta.get("tiles", "?"))


def learned_form(make_plan, dms, chunks, pulses, p, out, steps, plain_ms, plan_kw=None):
    """Learned proposal on the same stream: power tile + network + coherent
    processing of the top 10% of DM trials (full sweep if the proposal falls back).
    Its plan keeps compact records, so the visibilities produced and fetched are
    those of the proposed DMs only (the plain sweep's full records would carry
    zeros for every other DM).  Returns speedup over the plain sweep and the
    recall of the injected pulses."""
    import math

    import numpy as np
    import torch

    from paper_1109_3186_amd.proposal import Proposal, load_weights
    wpath = os.path.join(ROOT, "paper_1109_3186_amd", "proposal_weights.npz")
    full = torch.cat(chunks, dim=-1).contiguous()
    plan = make_plan(compact_records=True, **(plan_kw or {}))
    plan.set_dm_trials(dms)
    blocking = blocking_desc(plan.layout())
    prop = Proposal(plan, load_weights(wpath), budget=0.1)
    prec, wmeta = prop.net.precision, weights_provenance(wpath)

    def step():
        plan.reset_stream()
        mask, scores, fb = prop.select(full)
        plan.set_active_dms(mask)
        for i, ch in enumerate(chunks):
            plan.process_block(ch, flush=(i == len(chunks) - 1))
            plan.fetch(out=out)
        return mask, fb

    step()
    torch.cuda.synchronize()
    plan.set_profiling(True)
    t0 = time.perf_counter()
    for _ in range(steps):
        mask, fb = step()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    prof = plan.profile()
    plan.set_profiling(False)
    # the selection alone (tile, network, device top-k and the mask's copy), outside the timed steps
    t0 = time.perf_counter()
    for _ in range(steps):
        prop.select(full)
    torch.cuda.synchronize()
    select_ms = (time.perf_counter() - t0) * 1e3 / steps
    dstep = p["dm_max"] / p["n_dm"]
    hits = [int(mask[math.floor(q["dm"] / dstep)] or mask[min(math.ceil(q["dm"] / dstep), p["n_dm"] - 1)])
            for q in pulses]
    prop.close()
    plan.close()
    del full
    log("learned: %.1f ms/step (plain %.1f), %d active DMs, fallback %s, recall %d/%d" % (
        ms, plain_ms, int(mask.sum()), fb, sum(hits), len(hits)))
    return {"speedup": plain_ms / ms, "ms_per_step": ms, "active_dms": int(mask.sum()), "n_dm": p["n_dm"],
            "fallback": bool(fb), "recall": sum(hits) / len(hits), "pulses": len(hits),
            "network": "%s convolutions, weights %s" % (prec, wmeta), "select_ms": round(select_ms, 2),
            "blocking": blocking,
            "kernels_ms": {k: round(v["time_ms"] / steps, 1) for k, v in prof.items()},
            "launches": {k: v["launches"] // steps for k, v in prof.items()},
            "note": "tile + network + active-DM sweep on the same stream, records of the proposed DMs only; "
                    "recall = injected pulses whose DM trial "
                    "(either neighbour) is active"}


def recall_study(dev, n_streams=100, seed0=5000, log_every=10):
    """Voltage-level recall of the learned proposal over n_streams streams of the
    36-antenna workload's shape (10 pulses each: S/N 20, 100 us, random DM, time
    and position; seeds seed0 + i): power tile + network + device top-k alone, with
    the full sweep as the judge of its misses only.  Also compares each stream's
    voltage-generated tile with the power-model tile of the same pulses (the
    shortcut the network was trained on): the pulses' standardised peak heights and
    the standard deviation of the tile away from them."""
    import math

    import numpy as np
    import torch

    import synth
    from paper_1109_3186_amd import Plan
    from paper_1109_3186_amd.proposal import Proposal, load_weights
    p0 = synth.c1_params()
    fc = synth.chan_freqs(p0["f_lo"], p0["n_chan"], p0["f_s"])
    dms = synth.dm_grid(p0["n_dm"], p0["dm_max"])
    dstep = p0["dm_max"] / p0["n_dm"]
    wpath = os.path.join(ROOT, "paper_1109_3186_amd", "proposal_weights.npz")
    plan = Plan(p0["m_ant"], fc, p0["f_s"], p0["dump_len"], max_block_samples=1 << 18, in_dtype="ci8",
                compact_records=True)
    plan.set_dm_trials(dms)
    prop = Proposal(plan, load_weights(wpath), budget=0.1)
    network = "%s convolutions, weights %s" % (prop.net.precision, weights_provenance(wpath))
    gen = torch.Generator(device=dev)
    gen.manual_seed(seed0)
    rng = np.random.Generator(np.random.PCG64(seed0))
    hits = tot = fallbacks = 0
    missed = []
    peaks_v, peaks_m, sd_v, sd_m = [], [], [], []
    t0 = time.time()

    def zscore(t):
        t = t.double()
        return ((t - t.mean()) / t.std()).cpu().numpy()

    for i in range(n_streams):
        p = dict(p0, seed=seed0 + i)
        x, pulses, _, _ = synth.make_stream_device(p, dev)
        mask, _, fb = prop.select(x)
        del x
        fallbacks += int(fb)
        zv = zscore(prop.tile)
        power, _, _ = synth.power_batch(p, 1, 32, rng, gen, dev, pulses_given=[pulses])
        zm = zscore(plan.tiles_from_power(power, 32, 1024, 1024)[0])
        del power
        keep = np.ones(zv.shape, bool)
        for q in pulses:
            d0 = q["dm"] / dstep
            hit = bool(mask[math.floor(d0)] or mask[min(math.ceil(d0), p0["n_dm"] - 1)])
            tot += 1
            hits += int(hit)
            if not hit:
                missed.append((i, q))
            r, b = int(round(d0)), (q["n0"] + q["width"] // 2) // 1024
            rs, bs = slice(max(r - 2, 0), r + 3), slice(max(b - 2, 0), b + 3)
            peaks_v.append(float(zv[rs, bs].max()))
            peaks_m.append(float(zm[rs, bs].max()))
            keep[max(r - 12, 0):r + 13, :] = False
        sd_v.append(float(zv[keep].std()))
        sd_m.append(float(zm[keep].std()))
        if (i + 1) % log_every == 0:
            log("recall study: %d streams, %d/%d pulses kept, %d fallbacks, %.0f s" % (
                i + 1, hits, tot, fallbacks, time.time() - t0))
    prop.close()
    plan.close()
    torch.cuda.empty_cache()
    # the full sweep judges each miss: is the pulse found within one trial of its DM
    # by the autocorrelation power at the dump where each trial places it?
    judged = []
    if missed:
        full = Plan(p0["m_ant"], fc, p0["f_s"], p0["dump_len"], max_block_samples=1 << 18, in_dtype="ci8")
        full.set_dm_trials(dms)
        lay = full.layout()
        shift = lay["shift"].reshape(p0["n_chan"], p0["n_dm"])
        iu, ju = np.triu_indices(p0["m_ant"])
        auto_idx = torch.tensor(np.nonzero(iu == ju)[0], device=dev)
        for i in sorted({i for i, _ in missed}):
            x, _, _, _ = synth.make_stream_device(dict(p0, seed=seed0 + i), dev)
            full.reset_stream()
            pw = []
            for s0 in range(0, p0["samples"], 1 << 18):
                full.process_block(x[..., 2 * s0:2 * (s0 + (1 << 18))].contiguous(),
                                   flush=s0 + (1 << 18) >= p0["samples"])
                _, nd, vis = full.fetch()
                if nd:
                    pw.append(vis.view(nd, -1, lay["n_baselines"]).index_select(2, auto_idx).real.sum(dim=2)
                              .cpu().numpy())
            del x
            pw = np.concatenate(pw).reshape(-1, p0["n_chan"], p0["n_dm"])
            for j, q in missed:
                if j != i:
                    continue
                score = np.zeros(p0["n_dm"])
                for d in range(p0["n_dm"]):
                    m = (q["n0"] + q["width"] // 2 + shift[:, d]) // p0["dump_len"]
                    ok = m < pw.shape[0]
                    score[d] = pw[m[ok], np.nonzero(ok)[0], d].sum()
                judged.append({"stream": i, "dm": q["dm"], "sweep_finds": bool(abs(np.argmax(score) - q["dm"] / dstep)
                                                                                <= 1.0 + 1e-9)})
        full.close()
    recoverable = tot - sum(1 for j in judged if not j["sweep_finds"])
    pv, pm = np.array(peaks_v), np.array(peaks_m)
    rec = {"streams": n_streams, "pulses": tot, "kept": hits, "recall": hits / tot,
           "recall_of_sweep_recoverable": hits / max(recoverable, 1), "misses_judged_by_full_sweep": judged,
           "fallbacks": fallbacks, "seconds": round(time.time() - t0, 1), "network": network,
           "tile_validation": {"peak_z_voltage_median": round(float(np.median(pv)), 3),
                               "peak_z_power_model_median": round(float(np.median(pm)), 3),
                               "peak_ratio_median": round(float(np.median(pv / pm)), 4),
                               "peak_ratio_p10_p90": [round(float(np.quantile(pv / pm, 0.1)), 4),
                                                      round(float(np.quantile(pv / pm, 0.9)), 4)],
                               "noise_sd_voltage": round(float(np.mean(sd_v)), 4),
                               "noise_sd_power_model": round(float(np.mean(sd_m)), 4),
                               "tiles": n_streams}}
    log("recall study: %d/%d pulses kept (%.4f), %d misses judged by the full sweep, tiles: %s" % (
        hits, tot, hits / tot, len(judged), rec["tile_validation"]))
    return rec


def run_chirp(args, dev):
    """The Chirpolator pre-integrator (Sec. 3.2, App. A.3) on one complex baseband
    stream: 36 antennas (630 pairs), 2^22 samples of unit-variance noise, sliding
    DFT of length N = 2^16 sampled every L = 1024 samples, bins -100..100 (the
    paper's k0,max ~ 100 for the longest baselines).  One step = one call over the
    whole stream (partial DFTs of every block, then the block CIC)."""
    import numpy as np
    import torch

    from paper_1109_3186_amd import Chirp
    M, n, N, L, kmax = 36, 1 << 22, 1 << 16, 1024, 100
    g = torch.Generator(device=dev)
    g.manual_seed(1109)
    volts = torch.randn((M, n), dtype=torch.complex64, device=dev, generator=g)
    c = Chirp(M, N, L, kmax, max_samples=n)
    shape = c.output_shape(n)
    out = torch.empty(shape, dtype=torch.complex64, device=dev)
    for _ in range(args.warmup):
        c.preintegrate(volts, out=out)
    torch.cuda.synchronize()
    t0e, t1e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    t0e.record()
    for _ in range(args.steps):
        c.preintegrate(volts, out=out)
    t1e.record()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / args.steps
    ev_ms = t0e.elapsed_time(t1e) / args.steps
    pairs, bins = shape[1], shape[2]
    nb = n // L
    units = pairs * nb * L * bins
    value = units / (ms / 1e3)
    # bins k and -k share their four products (App. A.3, Eqs. fpos, fneg): four FMAs
    # per (pair, sample, k > 0), two for k = 0
    flops = 2.0 * pairs * nb * L * (4 * kmax + 2)
    tf = flops / (ev_ms / 1e3) / 1e12
    # per-pair bin budgets from the array geometry: 36 antennas in a 3 km-radius disk,
    # budget ceil(kmax b_pq / b_max) (the tone of a pair sits at k0 = B tau, tau <= b / c)
    import synth
    pos = synth.antenna_positions(np.random.Generator(np.random.PCG64(36)), M, 3000.0)
    blen = np.array([np.hypot(*(pos[p] - pos[q])) for p in range(M) for q in range(p + 1, M)])
    budgets = np.minimum(kmax, np.ceil(kmax * blen / blen.max())).astype(np.int32)
    c.set_pair_bins(budgets)
    for _ in range(args.warmup):
        c.preintegrate(volts, out=out)
    torch.cuda.synchronize()
    tb = time.perf_counter()
    for _ in range(args.steps):
        c.preintegrate(volts, out=out)
    torch.cuda.synchronize()
    ms_budget = (time.perf_counter() - tb) * 1e3 / args.steps
    c.set_pair_bins(None)
    budget_rec = {"mean_bins": round(float(np.mean(2 * budgets + 1)), 1), "ms": round(ms_budget, 2),
                  "speedup": round(ms / ms_budget, 3)}
    c.close()
    image_rec = image_leg(args, dev, out, pos, N, L, kmax)
    log("chirpolator: %.1f ms/step, %.3e pair-sample-bins/s, %.1f TFLOP/s; with per-pair budgets (mean %.1f of %d "
        "bins) %.1f ms" % (ms, value, tf, budget_rec["mean_bins"], 2 * kmax + 1, ms_budget))
    # the bank of lengths N0 d, d = 1..8 (N0 = N / 8), with the factorisation, against
    # the same eight lengths computed directly one by one
    import math

    from paper_1109_3186_amd import ChirpBank
    n0, n_len = N // 8, 8

    def timed(run):
        for _ in range(args.warmup):
            run()
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(args.steps):
            run()
        torch.cuda.synchronize()
        return (time.perf_counter() - t) * 1e3 / args.steps

    bank = ChirpBank(M, n0, n_len, L, kmax, max_samples=n)
    _, _, total = bank.layout(n)
    bout = torch.empty(total, dtype=torch.complex64, device=dev)
    ms_bank = timed(lambda: bank.run(volts, out=bout))
    bank.close()
    del bout
    ms_direct = 0.0
    for d in range(1, n_len + 1):
        cd = Chirp(M, n0 * d, L, kmax, max_samples=n)
        od = torch.empty(cd.output_shape(n), dtype=torch.complex64, device=dev)
        ms_direct += timed(lambda: cd.preintegrate(volts, out=od))
        cd.close()
        del od
    frac = sum(1 for d in range(1, n_len + 1) for kk in range(-kmax, kmax + 1) if math.gcd(abs(kk), d) > 1) / (
        n_len * (2 * kmax + 1))
    log("chirpolator bank of %d lengths: %.1f ms against %.1f ms direct (%.1f %% of bins factorised)" % (
        n_len, ms_bank, ms_direct, 100 * frac))
    bank_rec = {"n0": n0, "lengths": n_len, "ms_bank": round(ms_bank, 2), "ms_direct": round(ms_direct, 2),
                "speedup": round(ms_direct / ms_bank, 3), "factorised_fraction": round(frac, 4)}
    cpu = None
    if not args.no_cpu_baseline:
        # the FP64 oracle on one pair over the first 2048 blocks, one thread
        from threadpoolctl import threadpool_limits

        from oracle import chirpolator as och
        nbs = 2048   # about 10 s of oracle work
        s01 = volts[:2, :nbs * L].cpu().numpy().astype(np.complex128)
        with threadpool_limits(1):
            tc = time.perf_counter()
            och.block_cic(och.block_partial_dft(och.mix(s01, 0, 1), N, L, och.bins(kmax)), N, L)
            tc = time.perf_counter() - tc
        cpu = {"value": nbs * L * bins / tc, "unit": "pair-samples*bins/s", "cores": 1, "kind": "oracle",
               "sample": "pair (0, 1), first %d blocks, all %d bins, FP64 numpy on one thread, %.1f s" % (
                   nbs, bins, tc)}
        log("oracle slice: %.1f s" % tc)
    rec = {"metric": "pair-samples x DFT bins/s pre-integrated (Chirpolator)", "value": value,
           "unit": "pair-samples*bins/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
           "data": "synthetic",
           "config": {"workload": "Chirpolator pre-integrator: 36 ant (630 pairs) x 2^22 cf32 samples, N 2^16, "
                                  "L 1024, bins -100..100", "n_ant": M, "samples": n, "fft_len": N, "block_len": L,
                      "kmax": kmax, "parallelism": "none (1 GPU)"},
           "roofline": {"bound": "mfma", "achieved": round(tf, 2), "peak": PEAKS["fp32_mfma_tflops"],
                        "unit": "TFLOP/s", "frac": round(tf / PEAKS["fp32_mfma_tflops"], 4), "traffic": None,
                        "kernel": "partial DFT (FP32 MFMA) + block CIC (one call)", "avg_call_ms": round(ev_ms, 3)},
           "cpu_baseline": cpu, "bank": bank_rec, "pair_budgets": budget_rec, "image": image_rec}
    print(json.dumps(rec), flush=True)


def image_leg(args, dev, bins, pos2d, N, L, kmax):
    """The post-integrator image (Sec. 3.3, 3.4, App. A.1) on the pre-integrator's
    output: 256 x 256 directions over +-0.01 in l and m (16 x 16 tiles), F = 2, one
    image every 16 windows (4 per window length), the 36-antenna disk with heights
    of +-20 m; the chirp rate puts the longest baseline's tone at bin kmax - F at
    the field's corner.  Timed with HIP events on the launch stream; the weights
    are made once per plan, outside the timed region."""
    import numpy as np
    import torch

    import synth
    from paper_1109_3186_amd import Image
    F, n_side, lmax, w_step, f_s = 2, 256, 0.01, 16, 1e6
    M = pos2d.shape[0]
    heights = np.random.Generator(np.random.PCG64(37)).uniform(-20.0, 20.0, M)
    ant = np.concatenate([pos2d, heights[:, None]], axis=1)
    b_max = max(np.linalg.norm(ant[p] - ant[q]) for p in range(M) for q in range(p + 1, M))
    fdot = (kmax - F) * f_s * 299792458.0 / (N * b_max * lmax * np.sqrt(2.0))
    pix = synth.direction_grid(lmax, n_side)
    h = Image(ant, pix, fdot, f_s, N, L, kmax, F)
    n_img = h.output_count(bins.shape[0], w_step)
    for _ in range(args.warmup):
        h.run(bins, w_step=w_step)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(args.steps):
        h.run(bins, w_step=w_step)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    h.close()
    pairs = M * (M - 1) // 2
    terms = float(pix.shape[0]) * pairs * n_img * (2 * F + 1)
    tf = 8.0 * terms / (ms / 1e3) / 1e12   # one complex multiply-add per tap
    log("image: %d directions x %d images, F %d: %.2f ms, %.1f TFLOP/s" % (pix.shape[0], n_img, F, ms, tf))
    rec = {"directions": int(pix.shape[0]), "images": int(n_img), "half_width": F, "w_step": w_step,
           "ms_per_call": round(ms, 3), "direction_pair_images_per_s": pix.shape[0] * pairs * n_img / (ms / 1e3),
           "roofline": {"bound": "alu", "achieved": round(tf, 2), "peak": PEAKS["fp32_vector_tflops"],
                        "unit": "TFLOP/s", "frac": round(tf / PEAKS["fp32_vector_tflops"], 4),
                        "traffic": measured_traffic("image", "chirp", IMAGE_SOURCES), "kernel": "k_image"}}
    if not args.no_cpu_baseline:
        from threadpoolctl import threadpool_limits

        from oracle import imaging as oim
        sub = pix[:384]   # about 10 s of oracle work
        rows = bins[:1].cpu().numpy().astype(np.complex128)
        with threadpool_limits(1):
            tc = time.perf_counter()
            oim.image(rows, ant, sub, fdot, f_s, N, L, kmax, F)
            tc = time.perf_counter() - tc
        rec["cpu_baseline"] = {"value": sub.shape[0] * pairs / tc, "unit": "direction-pair-images/s", "cores": 1,
                               "kind": "oracle", "sample": "%d directions x 1 image, FP64 numpy on one thread, "
                                                           "%.1f s" % (sub.shape[0], tc)}
    return rec


def run_incoherent(args, dev):
    """Classical incoherent dedispersion (Sec. 2.3.1) of a power-beam spectrogram
    (Sec. 2.4.1): 1024 channels over 1.2-1.5 GHz (channel 0 highest), 2^18 samples of
    uniform random power, 1024 trials.  Brute force: DMs 0..1000 evenly, delays from
    Eq. dmdelay with the sample time that makes the largest delay 1023 samples.  Tree:
    its 1024 linear sweeps (delay 0..1023 across the band), the same span.  One step
    = one call of each; HIP events on the launch stream."""
    import numpy as np
    import torch

    from paper_1109_3186_amd import incoherent_dedisperse, incoherent_delays, tree_dedisperse
    C, T, D, k_dm = 1024, 1 << 18, 1024, 4.148808e15
    f = 1.5e9 - (0.3e9 / C) * (np.arange(C) + 0.5)
    dms = np.linspace(0.0, 1000.0, D)
    t_samp = k_dm * 1000.0 * (1.0 / f.min() ** 2 - 1.0 / f.max() ** 2) / 1023.0
    dl_h = incoherent_delays(f, t_samp, dms, k_dm)
    g = torch.Generator(device=dev)
    g.manual_seed(1113)
    power = torch.rand((C, T), dtype=torch.float32, device=dev, generator=g)
    dl = torch.from_numpy(dl_h).to(dev)
    n_out = T - int(dl_h.max())
    out = torch.empty((C, T), dtype=torch.float32, device=dev)
    work = torch.empty_like(out)

    def timed(run):
        for _ in range(args.warmup):
            run()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(args.steps):
            run()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / args.steps

    ms_tree = timed(lambda: tree_dedisperse(power, out=out, work=work))
    ms_brute = timed(lambda: incoherent_dedisperse(power, dl, n_out))
    tree_units = C * T * C / (ms_tree / 1e3)
    brute_units = C * n_out * D / (ms_brute / 1e3)
    # tree: the fused first five stages read and write every row once, and so does
    # each later pass of two stages (one alone if their count is odd; each input
    # row feeds four output rows, read once through L2)
    stages = int(np.log2(C))
    staged = 8.0 * C * T * (1 + (stages - 5 + 1) // 2)
    gbs = staged / (ms_tree / 1e3) / 1e9
    log("incoherent: tree %.2f ms (%.3e units/s, %.0f GB/s staged); brute force %.2f ms (%.3e units/s)" % (
        ms_tree, tree_units, gbs, ms_brute, brute_units))
    cpu = None
    if not args.no_cpu_baseline:
        from threadpoolctl import threadpool_limits

        from oracle import incoherent as oinc
        # the whole tree workload (about 10 s of oracle work)
        sub = power.cpu().numpy().astype(np.float64)
        with threadpool_limits(1):
            tc = time.perf_counter()
            oinc.tree(sub)
            tc = time.perf_counter() - tc
        del sub
        cpu = {"value": C * T * C / tc, "unit": "channel-samples*trials/s", "cores": 1, "kind": "oracle",
               "sample": "the whole workload: tree over %d channels x %d samples (%d sweeps), FP64 numpy on one "
                         "thread, %.1f s" % (C, T, C, tc)}
    rec = {"metric": "channel-samples x trials/s, tree incoherent dedispersion", "value": tree_units,
           "unit": "channel-samples*trials/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": ms_tree, "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
           "data": "synthetic",
           "config": {"workload": "incoherent dedispersion: 1024 ch x 2^18 samples, 1024 trials", "n_chan": C,
                      "samples": T, "trials": D, "parallelism": "none (1 GPU)"},
           "roofline": {"bound": "hbm", "achieved": round(gbs, 1), "peak": PEAKS["hbm_gbs"], "unit": "GB/s",
                        "frac": round(gbs / PEAKS["hbm_gbs"], 4),
                        "traffic": measured_traffic("tree", "incoherent", INCOHERENT_SOURCES),
                        "kernel": "k_tree_fused + k_tree_stage2 + k_tree_stage (one call)"},
           "cpu_baseline": cpu,
           "brute_force": {"ms_per_call": round(ms_brute, 3), "units_per_s": brute_units, "n_out": n_out,
                           "adds_per_s": C * n_out * D / (ms_brute / 1e3),
                           "tree_speedup_per_trial_sample": round(tree_units / brute_units, 1)}}
    print(json.dumps(rec), flush=True)


def run_chimg(args, dev):
    """The Chimageator (Sec. 4) on a uniform linear array of 64 antennas: 2^22
    unit-variance complex samples, blocks of L = 64 samples (65 536 blocks), a
    128-bin spatial DFT, and trajectory sums for 256 trials (end bins -32..31 x
    durations 64, 128, 256, 512 blocks) from every start block.  One step = the
    pre-integrator call + the trajectory call; HIP events on the launch stream."""
    import numpy as np
    import torch

    from paper_1109_3186_amd import chimg_preintegrate, chimg_trajectories
    M, n, L, n_s = 64, 1 << 22, 64, 128
    g = torch.Generator(device=dev)
    g.manual_seed(1114)
    volts = torch.randn((M, n), dtype=torch.complex64, device=dev, generator=g)
    trials = [(float(ke), tb) for tb in (64, 128, 256, 512) for ke in range(-32, 32)]
    ke = [t[0] for t in trials]
    tb = [t[1] for t in trials]

    def timed(run):
        for _ in range(args.warmup):
            run()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(args.steps):
            run()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / args.steps

    y = chimg_preintegrate(volts, L, n_s)
    ms_pre = timed(lambda: chimg_preintegrate(volts, L, n_s))
    ms_traj = timed(lambda: chimg_trajectories(y, M, L, ke, tb))
    # the same number of trials as 64 gradients x 4 durations: one pass per gradient
    # (partial sums) against the 256 trajectories summed separately
    from paper_1109_3186_amd import chimg_gradient_sums
    grads = [ke_ / 512.0 for ke_ in range(-32, 32)]
    lens = [64, 128, 256, 512]
    ms_grad = timed(lambda: chimg_gradient_sums(y, M, L, grads, lens))
    ms_sep = timed(lambda: chimg_trajectories(y, M, L, [g_ * t_ for t_ in lens for g_ in grads],
                                              [t_ for t_ in lens for _ in grads]))
    nb = n // L
    macs = nb * L * M * (M - 1) / 2.0                  # gridded products per call
    tf = 8.0 * macs / (ms_pre / 1e3) / 1e12
    gathers = sum(max(0, nb - t + 1) * t for t in tb)
    log("chimg: pre %.2f ms (%.1f TFLOP/s of products), trajectories %.2f ms (%.3e gathers/s); "
        "gradient partial sums %.2f ms against %.2f ms separately" % (
            ms_pre, tf, ms_traj, gathers / (ms_traj / 1e3), ms_grad, ms_sep))
    rec = {"metric": "antenna-samples/s through the Chimageator pre-integrator", "value": M * n / (ms_pre / 1e3),
           "unit": "antenna-samples/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": ms_pre + ms_traj, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f32", "data": "synthetic",
           "config": {"workload": "Chimageator: 64-antenna uniform line, 2^22 samples, L 64, 128 bins, 256 trials",
                      "n_ant": M, "samples": n, "block_len": L, "n_bins": n_s, "trials": len(trials),
                      "parallelism": "none (1 GPU)"},
           "roofline": {"bound": "mfma", "achieved": round(tf, 2), "peak": PEAKS["fp32_mfma_tflops"],
                        "unit": "TFLOP/s", "frac": round(tf / PEAKS["fp32_mfma_tflops"], 4),
                        "traffic": measured_traffic("pre", "chimg", CHIMG_SOURCES),
                        "kernel": "k_pre_mfma (pair products on FP32 MFMA + spatial DFT)"},
           "cpu_baseline": chimg_cpu_baseline(args, volts, L, n_s),
           "trajectories": {"ms_per_call": round(ms_traj, 3), "gathers_per_s": gathers / (ms_traj / 1e3),
                            "trials": len(trials)},
           "gradient_sums": {"gradients": len(grads), "durations": lens, "ms_per_call": round(ms_grad, 3),
                             "separate_ms": round(ms_sep, 3), "speedup": round(ms_sep / ms_grad, 2)}}
    print(json.dumps(rec), flush=True)


def chimg_cpu_baseline(args, volts, L, n_s):
    """The FP64 oracle's Chimageator pre-integrator on the first 32768 blocks (about
    10 s), one thread."""
    if args.no_cpu_baseline:
        return None
    import numpy as np
    from threadpoolctl import threadpool_limits

    from oracle import chimageator as ocg
    nb = 32768
    s = volts[:, :nb * L].cpu().numpy().astype(np.complex128)
    with threadpool_limits(1):
        tc = time.perf_counter()
        ocg.spatial_dft(ocg.grid_blocks(s, L), n_s)
        tc = time.perf_counter() - tc
    return {"value": s.shape[0] * nb * L / tc, "unit": "antenna-samples/s", "cores": 1, "kind": "oracle",
            "sample": "first %d blocks of %d samples, all %d antennas, FP64 numpy on one thread, %.2f s" % (
                nb, L, s.shape[0], tc)}


def run_c3(args, dev):
    print(json.dumps(c3_measure(dev, args.steps, args.warmup, args.corr, args.autotune, args.passes)), flush=True)


def c3_one_step(dev):
    """One timed step of the 256-antenna workload (after one warm-up step), for the
    default run's JSON line."""
    rec = c3_measure(dev, 1, 1, "f32", False, 0)
    keep = ("value", "unit", "ms_per_step", "steps", "warmup", "dtype", "config")
    out = {k: rec[k] for k in keep}
    out["dominant"] = {k: rec["roofline"][k] for k in ("bound", "achieved", "peak", "unit", "frac", "kernel")}
    out["kernels_ms_per_step"] = {k: v["ms_per_step"] for k, v in rec["roofline"]["kernels"].items()}
    return out


def c1_schedule(p, full_fc, dms, corr, chunk, measure=False):
    """Plan options of the 36-antenna workload: the autotuner's choice for the whole
    64-channel workload (also when only some channels run, so that counter runs
    see the headline's launch shapes), from the committed cache, or measured now
    (measure=True); the automatic schedule without an entry.  Returns (plan
    keyword arguments, a description)."""
    from paper_1109_3186_amd import autotune
    targs = (p["m_ant"], full_fc, p["f_s"], p["dump_len"], [dms] * len(full_fc))
    tuned = (autotune.tune(*targs, corr_dtype=corr, max_block=chunk, log=log) if measure
             else autotune.cached(*targs, corr_dtype=corr, max_block=chunk))
    if not tuned:
        key, desc = autotune.workload_key(*targs, corr, "ci8", chunk)
        log("no tuned entry for key %s (device %r): automatic schedule" % (key, desc["device"]))
        return {}, {"source": "automatic"}
    log("tuned (%s): cost model inverse %s ps, forward %s ps per point (N 2^8..2^18), wave %d group %d" % (
        tuned["source"], [round(v, 2) for v in tuned["cost_ps"][0]],
        [round(v, 2) for v in tuned["cost_ps"][1]], tuned["wave_units"], tuned["dm_group"]))
    return autotune.plan_kwargs(tuned), {"source": "autotuned (%s)" % tuned["source"],
                                         "wave_units": tuned["wave_units"], "dm_group": tuned["dm_group"]}


def c3_setup(dev, corr, use_autotune, n_passes):
    """The 256-antenna workload's stream (on the device) and its plan in the
    configuration c3_measure times: every channel's DM list cut into `passes`
    contiguous windows, compact records holding one window's (channel, DM) pairs.
    Returns a dict with p, x, fc, dms, plan, lay, passes, windows, masks, out."""
    import math

    import numpy as np
    import torch

    import synth
    from paper_1109_3186_amd import Plan, autotune

    p = synth.c3_params()
    t0 = time.time()
    x, pulses, fc, pos = synth.make_stream_device(p, dev)
    torch.cuda.synchronize()
    torch.cuda.empty_cache()  # the generator's temporaries go back to the device for the plan
    log("C3 input built in %.1f s" % (time.time() - t0))
    s, L, M = p["samples"], p["dump_len"], p["m_ant"]
    dms = [synth.dm_grid(n, p["dm_max"]) for n in p["n_dm"]]
    kw = {}
    if use_autotune:
        tuned = autotune.tune(M, fc, p["f_s"], L, dms, corr_dtype=corr, max_block=s, log=log)
        kw = autotune.plan_kwargs(tuned)
        log("tuned (%s): cost model inverse %s ps, forward %s ps per point (N 2^8..2^18), wave %d group %d" % (
            tuned["source"], [round(v, 2) for v in tuned["cost_ps"][0]], [round(v, 2) for v in tuned["cost_ps"][1]],
            tuned["wave_units"], tuned["dm_group"]))
    passes = n_passes or math.ceil(sum(p["n_dm"]) / 512)
    windows = [np.array_split(np.arange(n), passes) for n in p["n_dm"]]
    max_pairs = max(sum(len(windows[c][k]) for c in range(p["n_chan"])) for k in range(passes))
    ring = s // L + 2
    plan = Plan(M, fc, p["f_s"], L, max_block_samples=s, in_dtype="ci8", corr_dtype=corr, out_mode="packed",
                compact_records=True, max_record_pairs=max_pairs, ring_dumps=ring, **kw)
    for c, d in enumerate(dms):
        plan.set_dm_trials(d, chan=c)
    lay = plan.layout()
    log("C3 plan: %s, %d passes of <= %d pairs, ring %d dumps, %.1f GB device" % (
        blocking_desc(lay), passes, max_pairs, ring, lay["device_bytes"] / 1e9))
    out = torch.empty((ring, max_pairs * lay["n_baselines"]), dtype=torch.complex64, device=dev)
    masks = []
    for k in range(passes):
        mk = []
        for c, n in enumerate(p["n_dm"]):
            m = np.zeros(n, np.uint8)
            m[windows[c][k]] = 1
            mk.append(m)
        masks.append(mk)
    return {"p": p, "x": x, "fc": fc, "dms": dms, "plan": plan, "lay": lay, "passes": passes, "windows": windows,
            "masks": masks, "out": out}


def c3_pass(st, k):
    """Pass k of the 256-antenna step: the stream once through the plan with DM
    window k active; returns the number of dumps fetched into st["out"]."""
    plan = st["plan"]
    plan.reset_stream()
    for c in range(st["p"]["n_chan"]):
        plan.set_active_dms(st["masks"][k][c], chan=c)
    plan.process_block(st["x"], flush=True)
    _, nd, _ = plan.fetch(out=st["out"])
    return nd


def c3_measure(dev, steps, warmup, corr, use_autotune, n_passes):
    """The batched sparse-array workload: 256 antennas, 32 x 1 MHz channels at
    0.7-0.732 GHz, 2^18 ci8 samples, per-channel DM grids of 512..1536 trials over
    0-3000 (transform lengths 2^17 / 2^18, two-pass).  Its 2.26 TB of visibilities
    cannot be held, so one step runs the stream once per DM window: every channel's
    DM list is cut into `passes` contiguous windows, the plan's compact records
    hold one window's (channel, DM) pairs, and each pass fetches its dumps into a
    device buffer that the next pass reuses."""
    import torch

    st = c3_setup(dev, corr, use_autotune, n_passes)
    p, x, plan, lay, passes, out = st["p"], st["x"], st["plan"], st["lay"], st["passes"], st["out"]
    s, L, M = p["samples"], p["dump_len"], p["m_ant"]

    def step():
        return sum(c3_pass(st, k) for k in range(passes))

    for w in range(warmup):
        step()
        torch.cuda.synchronize()
        log("C3 warmup %d done" % w)
    plan.set_profiling(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        got = step()
        log("C3 step %d enqueued" % k)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    prof = plan.profile()
    plan.set_profiling(False)
    n_dumps = got // passes
    units = M * n_dumps * L * sum(p["n_dm"])
    value = units / (ms / 1e3)
    log("C3 per step: %.1f ms, %.3e units/s; kernels: %s" % (
        ms, value, {k: round(v["time_ms"] / steps, 1) for k, v in prof.items()}))
    roofline = roofline_of(prof, argparse.Namespace(workload="c3", corr=corr, steps=steps))
    rec = {
        "metric": METRIC, "value": value, "unit": UNIT, "n_gpus": 1, "steps": steps, "warmup": warmup,
        "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": corr, "data": "synthetic",
        "config": {"workload": "256 ant x 32 ch x 2^18 ci8 samples, 512..1536 DMs per channel 0-3000, "
                               "%s, 1 ms dumps, %d DM-window passes" % (blocking_desc(lay), passes),
                   "n_ant": M, "n_chan": p["n_chan"], "samples": s, "n_dm_total": int(sum(p["n_dm"])),
                   "dump_len": L, "passes": passes, "input": "ci8", "corr": corr,
                   "schedule": {"wave_units": lay["wave_units"], "dm_group": lay["dm_group"],
                                "autotuned": bool(use_autotune)}, "parallelism": "none (1 GPU)"},
        "roofline": roofline, "cpu_baseline": None, "learned": None,
    }
    plan.close()
    del x, out
    st.clear()
    torch.cuda.empty_cache()
    return rec


SAMPLED_PAIRS = [(0, 255), (31, 128), (63, 0), (63, 201)]


def run_stream(plan, chunks, out, pairs=None, lay=None):
    """One pass of the stream through a plan (reset, every chunk, fetch into `out`);
    with `pairs`, host copies of those (channel, DM) records.  Returns (dumps, kept)."""
    plan.reset_stream()
    got = 0
    keep = {k: [] for k in (pairs or [])}
    for i, ch in enumerate(chunks):
        plan.process_block(ch, flush=(i == len(chunks) - 1))
        _, nd, _ = plan.fetch(out=out)
        got += nd
        if pairs and nd:
            v = out[:nd].view(nd, -1, lay["n_baselines"])
            for (c, d) in pairs:
                keep[(c, d)].append(v[:, int(lay["record_pos"][lay["dm_offset"][c] + d])].cpu().numpy())
    import numpy as np
    return got, {k: np.concatenate(v) for k, v in keep.items()}


def error_table(kept, host, fc, dms, lay, p):
    """Normalised errors |dV_ij| / sqrt(V_ii V_jj) of sampled (channel, DM) records
    against the FP64 oracle (one thread per pair)."""
    from concurrent.futures import ThreadPoolExecutor

    import numpy as np
    from threadpoolctl import threadpool_limits

    import oracle
    from paper_1109_3186_amd import layout_blockings
    bl = layout_blockings(lay)
    iu, ju = np.triu_indices(p["m_ant"])

    def one(cd):
        c, d = cd
        ref = oracle.run_oracle(host[c][None], fc[c:c + 1], p["f_s"], [dms], p["dump_len"], [bl[c]], chans=[0],
                                dm_index=[d])[(0, d)]
        auto = ref[:, iu == ju].real
        norm = np.sqrt(auto[:, iu] * auto[:, ju])
        return d, (np.abs(kept[cd].astype(np.complex128) - ref) / norm).ravel()

    with threadpool_limits(limits=1), ThreadPoolExecutor(len(kept)) as ex:
        res = list(ex.map(one, list(kept)))
    e = np.concatenate([r for d, r in res if d != 0] or [np.zeros(1)])
    z = np.concatenate([r for d, r in res if d == 0] or [np.zeros(1)])
    return {"pairs": [list(k) for k in kept], "visibilities": int(e.size + z.size), "max_dm_gt0": float(e.max()),
            "p999_dm_gt0": float(np.quantile(e, 0.999)), "rms_dm_gt0": float(np.sqrt(np.mean(e ** 2))),
            "max_dm0": float(z.max()), "max": float(max(e.max(), z.max()))}


def precision_forms(forms, make_plan, dms, chunks, host, fc, p, steps):
    """The reduced-precision correlator inputs on the same stream: per form, one
    untimed pass whose sampled records give the error table against the FP64 oracle,
    then `steps` timed passes (library event timings per kernel kind)."""
    import torch
    res = {}
    for corr in forms:
        plan = make_plan(corr_dtype=corr)
        plan.set_dm_trials(dms)
        lay = plan.layout()
        out = torch.empty((lay["ring_dumps"], lay["record_elems"]), dtype=torch.complex64, device="cuda")
        _, kept = run_stream(plan, chunks, out, SAMPLED_PAIRS, lay)
        torch.cuda.synchronize()
        plan.set_profiling(True)
        t0 = time.perf_counter()
        for _ in range(steps):
            n_dumps, _ = run_stream(plan, chunks, out)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / steps
        prof = plan.profile()
        plan.set_profiling(False)
        lay = plan.layout()
        plan.close()
        del out
        units = p["m_ant"] * n_dumps * p["dump_len"] * p["n_chan"] * p["n_dm"]
        err = error_table(kept, host, fc, dms, lay, p)
        dd = prof.get("dedisperse", {"time_ms": 0.0, "flops": 0.0})
        rec = {"value": units / (ms / 1e3), "ms_per_step": ms, "steps": steps,
               "kernels_ms_per_step": {k: round(v["time_ms"] / steps, 1) for k, v in prof.items() if v["launches"]},
               "dedisperse_tflops": round(dd["flops"] / max(dd["time_ms"], 1e-9) / 1e9, 2),
               "scales": sorted(set(float(v) for v in lay["scale"])), "errors_vs_fp64_oracle": err}
        log("%s form: %.1f ms/step, %.3e units/s; error max %.3e (DM > 0 99.9%% %.3e, DM 0 %.3e)" % (
            corr, ms, rec["value"], err["max"], err["p999_dm_gt0"], err["max_dm0"]))
        res[corr] = rec
    return res


def roofline_of(prof, args, p=None, ms_step=None):
    """Roofline of the dominant kernel kind from the library's event timings.

    Dedispersion (A4: chirp multiply, inverse FFT, discard) runs on the FP32 vector
    units: achieved = its algorithmic FLOP per launch (5 N log2 N / V + 6 N / V per
    unit, times the V M units of each of the launch's (channel, DM, block) units) /
    its average launch duration, against the 157.3 TFLOP/s FP32 vector peak.  Beside
    it: the HBM rate from the committed FETCH_SIZE / WRITE_SIZE counters (`traffic`,
    bytes per launch; null if the kernel sources changed since), and the staged-byte
    model (a spectrum read per unit and antenna, the chirps, the voltages written),
    labelled as a model.  Correlator (A6, dominant at 256 antennas): MFMA, against
    the peak of its input format."""
    dom = max(prof, key=lambda k: prof[k]["time_ms"])
    d = prof[dom]
    n = max(d["launches"], 1)
    per_launch_s = d["time_ms"] / 1e3 / n
    tflops = d["flops"] / n / per_launch_s / 1e12
    traffic = measured_traffic(dom, args.workload)
    if dom == "correlate":
        peak = {"f32": PEAKS["fp32_mfma_tflops"], "f16": PEAKS["fp16_mfma_tflops"],
                "e4m3": PEAKS["fp8_mfma_tflops"]}[args.corr]
        r = {"bound": "mfma", "achieved": round(tflops, 2), "peak": peak, "unit": "TFLOP/s",
             "frac": round(tflops / peak, 4)}
    else:
        r = {"bound": "alu", "achieved": round(tflops, 2), "peak": PEAKS["fp32_vector_tflops"], "unit": "TFLOP/s",
             "frac": round(tflops / PEAKS["fp32_vector_tflops"], 4)}
        up = PEAKS["fp32_vector_unpacked_tflops"]
        r["unpacked_fp32"] = {"peak": round(up, 1), "frac": round(tflops / up, 4),
                              "note": "the FP32 FMA rate without packed instructions, which the library does not emit"}
        gbs = d["bytes"] / n / per_launch_s / 1e9
        r["staged_model"] = {"gbs": round(gbs, 1), "frac_of_hbm": round(gbs / PEAKS["hbm_gbs"], 4),
                             "note": "modelled bytes (8 N / V + b_y per unit), not measured"}
    r.update({"traffic": traffic, "kernel": dom, "avg_launch_ms": round(per_launch_s * 1e3, 4)})
    if traffic:
        r["hbm_counters"] = {"gbs": round(traffic / per_launch_s / 1e9, 1),
                             "frac": round(traffic / per_launch_s / 1e9 / PEAKS["hbm_gbs"], 4),
                             "source": "profiles/traffic_%s_%s.json" % (dom, args.workload)}
    if p is not None and ms_step:
        # the method's own minimum bytes: the input once and the visibilities out
        units = p["units"]
        alg = p["input_bytes"] + p["vis_bytes"]
        r["path_algorithmic_bytes"] = {"bytes_per_step": alg, "per_unit": round(alg / units, 4),
                                       "gbs": round(alg / (ms_step / 1e3) / 1e9, 1)}
    r["kernels"] = {k: {"ms_per_step": round(v["time_ms"] / args.steps, 2),
                        "launches_per_step": v["launches"] // args.steps,
                        "tflops": round(v["flops"] / max(v["time_ms"], 1e-9) / 1e9, 2),
                        "staged_gbs": round(v["bytes"] / max(v["time_ms"], 1e-9) / 1e6, 1)}
                    for k, v in prof.items() if v["launches"]}
    return r


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--corr", default="f32", choices=["f32", "f16", "e4m3"])
    ap.add_argument("--chunk", type=int, default=1 << 18, help="samples per process_block call")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-dms-per-thread", type=int, default=12,
                    help="DM trials per host thread in the oracle's timed slice")
    ap.add_argument("--forms", default="f16,e4m3",
                    help="reduced-precision correlator inputs measured after the main form (comma list, '' = none)")
    ap.add_argument("--form-steps", type=int, default=3, help="timed passes per reduced-precision form")
    ap.add_argument("--no-c3", action="store_true", help="skip the one-step 256-antenna leg of the default run")
    ap.add_argument("--recall-streams", type=int, default=100,
                    help="voltage streams of the learned proposal's recall study (10 pulses each; 0 = skip)")
    ap.add_argument("--no-learned", action="store_true", help="skip the learned-proposal measurement")
    ap.add_argument("--wave-units", type=int, default=0, help="schedule: units per wave (0 = automatic)")
    ap.add_argument("--dm-group", type=int, default=0, help="schedule: DMs per block group (0 = automatic)")
    ap.add_argument("--workload", default="c1", choices=["c1", "c3", "chirp", "incoherent", "chimg"],
                    help="c1: 36-antenna headline workload (default); c3: 256-antenna batched sparse array; "
                         "chirp: the Chirpolator pre-integrator and image; incoherent: classical incoherent "
                         "dedispersion of a power spectrogram (brute force and tree); chimg: the Chimageator on a "
                         "uniform linear array")
    ap.add_argument("--autotune", action="store_true",
                    help="tune the blocking cost model and schedule now if the cache has no entry for this device "
                         "and workload (without it: the committed cache's entry when there is one; the 256-antenna "
                         "leg only with it)")
    ap.add_argument("--passes", type=int, default=0, help="c3: DM-window passes (0 = ceil(sum D / 512))")
    ap.add_argument("--channels", type=int, default=0,
                    help="run only the first CHANNELS channels (a smaller workload for counter runs; 0 = all)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="before the steps, run one elementwise copy kernel of MIB MiB (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path (requested %d)" % args.gpus,
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import synth
    from paper_1109_3186_amd import Plan

    dev = torch.device("cuda:0")
    if args.workload == "c3":
        return run_c3(args, dev)
    if args.workload == "chirp":
        return run_chirp(args, dev)
    if args.workload == "incoherent":
        return run_incoherent(args, dev)
    if args.workload == "chimg":
        return run_chimg(args, dev)
    if args.copy_calibration:
        src = torch.ones(args.copy_calibration << 18, dtype=torch.float32, device=dev)
        dst = torch.mul(src, 1.0)  # reads and writes copy_calibration MiB each
        torch.cuda.synchronize()
        log("copy calibration: %d MiB read, %d MiB written by one elementwise kernel" % (
            args.copy_calibration, args.copy_calibration))
        del src, dst
    p = synth.c1_params()
    full_fc = synth.chan_freqs(p["f_lo"], p["n_chan"], p["f_s"])
    if args.channels:
        p["n_chan"] = min(args.channels, p["n_chan"])
    chunks, pulses, fc = build_input(p, dev, args.chunk)
    dms = synth.dm_grid(p["n_dm"], p["dm_max"])
    kw = {"wave_units": args.wave_units, "dm_group": args.dm_group}
    schedule = {"source": "automatic"}
    if not (args.wave_units or args.dm_group):
        kw, schedule = c1_schedule(p, full_fc, dms, args.corr, args.chunk, args.autotune)
    def make_plan(**extra):
        opts = dict(kw, corr_dtype=args.corr)
        opts.update(extra)
        return Plan(p["m_ant"], fc, p["f_s"], p["dump_len"], max_block_samples=args.chunk, in_dtype="ci8",
                    out_mode="packed", **opts)

    plan = make_plan()
    plan.set_dm_trials(dms)
    lay = plan.layout()
    log("plan: %s, V %d..%d, ring %d dumps, %.1f GB device, wave %d units, DM group %d" % (
        blocking_desc(lay), lay["dm_valid"].min(), lay["dm_valid"].max(), lay["ring_dumps"],
        lay["device_bytes"] / 1e9, lay["wave_units"], lay["dm_group"]))
    out = torch.empty((lay["ring_dumps"], lay["record_elems"]), dtype=torch.complex64, device=dev)

    def step():
        plan.reset_stream()
        got = 0
        for i, ch in enumerate(chunks):
            plan.process_block(ch, flush=(i == len(chunks) - 1))
            _, nd, _ = plan.fetch(out=out)
            got += nd
        return got

    for w in range(args.warmup):
        n_dumps = step()
        torch.cuda.synchronize()
        log("warmup %d done (%d dumps)" % (w, n_dumps))
    plan.set_profiling(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        n_dumps = step()
        log("step %d enqueued" % k)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = plan.profile()
    plan.set_profiling(False)
    ms = (t1 - t0) * 1e3 / args.steps
    units = p["m_ant"] * n_dumps * p["dump_len"] * p["n_chan"] * p["n_dm"]
    value = units / (ms / 1e3)
    log("per step: %.1f ms, %.3e units/s; kernels: %s" % (
        ms, value, {k: round(v["time_ms"] / args.steps, 1) for k, v in prof.items()}))

    path = {"units": units, "input_bytes": 2.0 * p["m_ant"] * p["n_chan"] * p["samples"],
            "vis_bytes": 8.0 * n_dumps * p["n_chan"] * p["n_dm"] * lay["n_baselines"]}
    roofline = roofline_of(prof, args, path, ms)
    learned = None
    if not args.no_learned:
        # one blocking class per channel: with a tenth of the trials active, each class's
        # forward transforms serve few DMs, and one 32768-point class measured fastest
        learned = learned_form(make_plan, dms, chunks, pulses, p, out, args.steps, ms,
                               plan_kw={"dm_classes": "single"})
    del out
    plan.close()
    c3 = None
    if not args.no_c3 and args.corr == "f32" and not args.channels:
        import gc
        gc.collect()
        torch.cuda.empty_cache()
        free, total = torch.cuda.mem_get_info()
        log("device memory before the 256-antenna leg: %.1f GB free of %.1f GB" % (free / 1e9, total / 1e9))
        c3 = c3_one_step(dev)
    if learned is not None and args.recall_streams > 0 and not args.channels:
        learned["recall_study"] = recall_study(dev, args.recall_streams)
    forms = None
    if args.forms and args.corr == "f32" and not args.channels:
        host = {c: np.concatenate([ch[c].cpu().numpy() for ch in chunks], axis=-1)
                for c in sorted({c for c, _ in SAMPLED_PAIRS})}
        forms = precision_forms([f for f in args.forms.split(",") if f], make_plan, dms, chunks, host, fc, p,
                                args.form_steps)
    cpu = None
    if not args.no_cpu_baseline:
        log("timing the oracle on a slice")
        cpu = cpu_baseline(chunks, fc, dms, lay, p, args.cpu_dms_per_thread)
    rec = {
        "metric": METRIC, "value": value, "unit": UNIT, "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": {"f32": "f32", "f16": "f16", "e4m3": "e4m3"}[args.corr], "data": "synthetic",
        "config": {"workload": "36 ant x %d ch x 2^20 ci8 samples, 256 DMs 0-2000, %s, 1 ms dumps"
                               % (p["n_chan"], blocking_desc(lay)),
                   "n_ant": p["m_ant"], "n_chan": p["n_chan"], "samples": p["samples"], "n_dm": p["n_dm"],
                   "dump_len": p["dump_len"], "fft_len": sorted(set(int(v) for v in lay["dm_fft_len"])),
                   "dm_classes": int(lay["n_classes"]), "chunk": args.chunk, "schedule": schedule,
                   "input": "ci8", "corr": args.corr, "parallelism": "none (1 GPU)"},
        "roofline": roofline, "cpu_baseline": cpu, "learned": learned, "precision_forms": forms, "c3_step": c3,
        "paper_context": PAPER_CONTEXT,
    }
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
