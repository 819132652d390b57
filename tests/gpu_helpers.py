"""Helpers shared by the GPU tests: run the HIP path through the C ABI and
compare its visibilities with the FP64 oracle."""
import sys

import numpy as np

import oracle


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def run_gpu(cfg, in_dtype="cf32", corr="f32", out_mode="packed", chunks=None, fft_len=None, mask=None,
            max_block=None, chan_scale=None, **plan_kw):
    """Run a whole stream through the library; returns (vis [dumps, record] complex64 numpy, layout)."""
    import torch

    from paper_1109_3186_amd import Plan

    x = cfg["volts"]
    m_ant = x.shape[1]
    s = x.shape[-1] // 2 if in_dtype == "ci8" else x.shape[-1]
    chunks = [s] if chunks is None else chunks
    assert sum(chunks) == s
    mb = max(chunks) if max_block is None else max_block
    dev = torch.device("cuda:0")
    fl = fft_len if fft_len is not None else (cfg.get("fft_len") or None)
    outs = []
    with Plan(m_ant, cfg["chan_freqs"], cfg["f_s"], cfg["dump_len"], max_block_samples=mb, in_dtype=in_dtype,
              corr_dtype=corr, out_mode=out_mode, fft_len=fl, chan_scale=chan_scale, **plan_kw) as p:
        for c, dms in enumerate(cfg["dm_lists"]):
            p.set_dm_trials(dms, chan=c)
        if mask is not None:
            for c, mk in enumerate(mask):
                p.set_active_dms(mk, chan=c)
        lay = p.layout()
        pos = 0
        for i, n in enumerate(chunks):
            if in_dtype == "ci8":
                part = np.ascontiguousarray(x[..., 2 * pos:2 * (pos + n)])
            else:
                part = np.ascontiguousarray(x[..., pos:pos + n])
            t = torch.from_numpy(part).to(dev)
            p.process_block(t, flush=(i == len(chunks) - 1))
            first, nd, vis = p.fetch()
            if nd:
                outs.append(vis.cpu().numpy())
            torch.cuda.synchronize()
            del t
            pos += n
        lay_end = p.layout()
    vis = np.concatenate(outs, axis=0) if outs else np.zeros((0, lay["record_elems"]), np.complex64)
    return vis, lay_end


def blockings(lay):
    """Per channel, the list of every DM's blocking (its class's) from a plan layout."""
    from paper_1109_3186_amd import layout_blockings
    return layout_blockings(lay)


def select(vis, lay, c, d):
    """Visibilities of (channel c, DM d) from fetched records (its record slot)."""
    nbl = lay["n_baselines"]
    o = int(lay["record_pos"][lay["dm_offset"][c] + d])
    assert o >= 0, "(channel %d, DM %d) is not stored in the records" % (c, d)
    return vis[:, o * nbl:(o + 1) * nbl]


def norm_error(got, ref, m_ant):
    """max |V_got - V_ref| / sqrt(V_ii V_jj) with the reference autocorrelations (packed layout)."""
    iu, ju = np.triu_indices(m_ant)
    auto = ref[:, iu == ju].real
    norm = np.sqrt(np.maximum(auto[:, iu] * auto[:, ju], 1e-300))
    return float(np.max(np.abs(got.astype(np.complex128) - ref) / norm)) if ref.size else 0.0


def compare_with_oracle(cfg, vis, lay, pairs=None, quant=None, scales=None):
    """Max normalised error over (channel, DM) pairs (all by default)."""
    m_ant = cfg["volts"].shape[1]
    bl = blockings(lay)
    worst = 0.0
    chans = sorted({c for c, _ in pairs}) if pairs else range(lay["n_chan"])
    for c in chans:
        ds = [d for cc, d in pairs if cc == c] if pairs else None
        ref = oracle.run_oracle(cfg["volts"], cfg["chan_freqs"], cfg["f_s"], cfg["dm_lists"], cfg["dump_len"], bl,
                                sideband=int(lay["sideband"]), quant=quant, scales=scales, chans=[c], dm_index=ds)
        for (cc, d), v in ref.items():
            got = select(vis, lay, cc, d)
            assert got.shape == v.shape, (got.shape, v.shape)
            worst = max(worst, norm_error(got, v, m_ant))
    return worst


def quant_errors(cfg, vis, lay, quant, scales, skip_dm0=True):
    """Normalised errors vs the emulating and the exact oracle, DM-0 trials apart."""
    m_ant = cfg["volts"].shape[1]
    bl = blockings(lay)
    emu, exact, dm0 = [], [], [np.zeros(0)]
    for c in range(lay["n_chan"]):
        rq = oracle.run_oracle(cfg["volts"], cfg["chan_freqs"], cfg["f_s"], cfg["dm_lists"], cfg["dump_len"], bl,
                               quant=quant, scales=scales, chans=[c])
        rx = oracle.run_oracle(cfg["volts"], cfg["chan_freqs"], cfg["f_s"], cfg["dm_lists"], cfg["dump_len"], bl,
                               chans=[c])
        iu, ju = np.triu_indices(m_ant)
        for (cc, d), vq in rq.items():
            got = select(vis, lay, cc, d).astype(np.complex128)
            vx = rx[(cc, d)]
            auto = vx[:, iu == ju].real
            norm = np.sqrt(auto[:, iu] * auto[:, ju])
            if skip_dm0 and cfg["dm_lists"][cc][d] == 0:
                dm0.append((np.abs(got - vx) / norm).ravel())
                continue
            emu.append((np.abs(got - vq) / norm).ravel())
            exact.append((np.abs(got - vx) / norm).ravel())
    return np.concatenate(emu), np.concatenate(exact), np.concatenate(dm0)


def _complex_volts(v):
    """[M, S] complex from complex input or [M, 2S] interleaved int8."""
    v = np.asarray(v)
    if np.iscomplexobj(v):
        return v.astype(np.complex128)
    return v[..., 0::2].astype(np.float64) + 1j * v[..., 1::2].astype(np.float64)


def tie_check(cfg, vis, lay, quant, scales, delta_rel=1e-4):
    """Reduced-precision cross visibilities against the oracle emulating the same
    rounding, with an allowance for rounding ties.  A scaled voltage component lying
    within delta of a rounding midpoint (delta = delta_rel x the channel and DM's RMS
    scaled component: the FP32 dedispersion's own error stays below it, by about an
    order of magnitude) may round to either neighbour on the GPU; such a tie can move
    V_ij (i < j) by at most the distance between its two candidates times the other
    voltage's magnitude (both flipping: plus the product of the two distances).
    Returns the normalised errors and allowances of every cross visibility (every
    channel, DM and dump), whether each belongs to a DM-0 trial, the
    autocorrelations' errors against the unrounded oracle, and the counts of tie
    components and of all components (DM > 0)."""
    m_ant = cfg["volts"].shape[1]
    bl = blockings(lay)
    iu, ju = np.triu_indices(m_ant)
    cross = iu != ju
    L = cfg["dump_len"]
    errs, allows, autos, dm0 = [], [], [], []
    n_tie = n_all = 0
    for c in range(lay["n_chan"]):
        x = _complex_volts(cfg["volts"][c])
        s = float(scales[c])
        ref = oracle.run_oracle(cfg["volts"], cfg["chan_freqs"], cfg["f_s"], cfg["dm_lists"], L, bl,
                                sideband=int(lay["sideband"]), quant=quant, scales=scales, chans=[c])
        for d, dm in enumerate(cfg["dm_lists"][c]):
            b = bl[c][d] if isinstance(bl[c], (list, tuple)) else bl[c]
            h = oracle.chirp(cfg["chan_freqs"][c], cfg["f_s"], b["fft_len"], dm, int(lay["sideband"]))
            y = oracle.dedisperse_stream(x, h, b["fft_len"], b["valid"], b["lead"])
            nd = y.shape[1] // L
            vs = y[:, :nd * L] * s
            delta = delta_rel * np.sqrt(np.mean(np.abs(vs) ** 2) / 2.0)
            q = oracle.quantize(vs, quant)
            lo = oracle.quantize(vs - delta * (1 + 1j), quant)
            hi = oracle.quantize(vs + delta * (1 + 1j), quant)
            dre, dim = np.abs(hi.real - lo.real), np.abs(hi.imag - lo.imag)
            if dm != 0:
                n_tie += int(np.count_nonzero(dre) + np.count_nonzero(dim))
                n_all += 2 * vs.size
            dq = np.hypot(dre, dim).reshape(m_ant, nd, L)
            aq = np.abs(q).reshape(m_ant, nd, L)
            allow = (np.einsum("ind,jnd->nij", dq, aq) + np.einsum("ind,jnd->nij", aq, dq)
                     + np.einsum("ind,jnd->nij", dq, dq)) / (s * s)
            v = ref[(c, d)]
            got = select(vis, lay, c, d).astype(np.complex128)
            assert got.shape == v.shape
            auto = v[:, iu == ju].real
            norm = np.sqrt(auto[:, iu] * auto[:, ju])
            e = np.abs(got - v) / norm
            errs.append(e[:, cross].ravel())
            allows.append((oracle.pack_upper(allow) / norm)[:, cross].ravel())
            autos.append(e[:, ~cross].ravel())
            dm0.append(np.full(errs[-1].size, dm == 0))
    return (np.concatenate(errs), np.concatenate(allows), np.concatenate(dm0), np.concatenate(autos), n_tie,
            n_all)
