"""Plain FP64 coherent dedispersion + cross-multiply + integrate-and-dump.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Notation follows Bannister & Cornwell (2011):
  DM        dispersion measure in pc cm^-3 (Sec. 2.1)
  K         the dispersion constant mu = e^2 / (2 pi m_e c) of Eq. dmdelay,
            here in s Hz^2 per pc cm^-3 (mu ~ 4.15 ms with frequencies in GHz)
  f_s       complex Nyquist sample rate = channel bandwidth (Sec. 3.2)
  s_p[n]    complex baseband voltage of antenna p (Sec. 3.2, Eq. chirp)
  x_pq      the mixed product s_p s_q^* (Sec. 3.2, Eq. xpq)
  L         integrate-and-dump length in samples (Sec. 5.1; the block length
            of the block partial DFT, Appendix A.3, Eq. block_cic)

Readings taken where the paper is silent (each is listed in the design doc):
  * the filter is exp(-2 pi i K DM f^2 / (f_c^2 (f_c + f))), the delay law of
    Eq. dmdelay turned into a transfer function with its constant and linear
    (channel-centre delay) terms dropped, as Sec. 2.1 drops them for the chirp;
  * bins follow the unnormalised forward DFT exp(-2 pi i k n / N) with the
    inverse scaled by 1/N, bin N/2 is -f_s/2, and the sideband sign maps a
    baseband offset f to the sky frequency f_c + sideband * f;
  * overlap-save blocks of N samples keep V = N - lead - trail outputs, V a
    multiple of L, lead/trail >= the early/late intra-channel smear;
  * V_ij = sum_n y_i[n] conj(y_j[n]) over whole dumps only; packed upper
    triangle including the autocorrelations.
"""

import math

import numpy as np

# Dispersion constant e^2 / (2 pi m_e c) in s Hz^2 cm^3 / pc (Sec. 2.1, the
# constant mu of Eq. dmdelay, ~4.15 ms for frequencies in GHz).
K_DM = 4.148808e15


def smear_samples(f_c, f_s, dm, k_dm=K_DM):
    """Intra-channel dispersion smear of channel centred at sky frequency f_c.

    Eq. dmdelay (Sec. 2.1) gives the delay between two sky frequencies as
    K DM (nu_2^-2 - nu_1^-2).  Relative to the channel centre, the top edge
    f_c + f_s/2 arrives ``early`` seconds before it and the bottom edge
    f_c - f_s/2 arrives ``late`` seconds after it.  Both are returned in
    samples (times f_s).
    """
    nu_hi = f_c + 0.5 * f_s
    nu_lo = f_c - 0.5 * f_s
    inv_c = 1.0 / (f_c * f_c)
    early = k_dm * dm * (inv_c - 1.0 / (nu_hi * nu_hi)) * f_s
    late = k_dm * dm * (1.0 / (nu_lo * nu_lo) - inv_c) * f_s
    return early, late


def blocking(f_c, f_s, dm_max, dump_len, fft_len=0, k_dm=K_DM):
    """Overlap-save blocking of one channel.

    The paper fixes no FFT length or overlap (Sec. 2.3.2 only says the
    voltages are convolved with the inverse ISM response).  Reading used here:
    half-overlap A = ceil(max(early, late)) samples at the largest DM of the
    channel; V = the largest multiple of L not above N - 2A; the discarded
    N - V samples are split lead = floor((N-V)/2) before and trail = rest after
    the kept range.  With fft_len = 0, N is the smallest power of two >= 256
    that keeps at least half of every block (V >= N/2).
    """
    early, late = smear_samples(f_c, f_s, dm_max, k_dm)
    a = int(math.ceil(max(early, late)))

    def kept(n):
        return dump_len * ((n - 2 * a) // dump_len)

    n = int(fft_len)
    if n == 0:
        n = 256
        while kept(n) < n // 2:
            n *= 2
    v = kept(n)
    if v < dump_len:
        raise ValueError("FFT length %d too short for smear %d and dump %d" % (n, 2 * a, dump_len))
    lead = (n - v) // 2
    return {"fft_len": n, "valid": v, "lead": lead, "trail": n - v - lead, "half_overlap": a}


def bin_offsets(n, f_s, sideband=1):
    """Sky-frequency offset from the channel centre of each DFT bin (Hz).

    Bin k of an N-point DFT at complex Nyquist rate f_s (Sec. 3.2: f_s = B)
    is at k f_s / N for k < N/2 and (k - N) f_s / N otherwise; a lower
    sideband flips the sign.
    """
    k = np.arange(n, dtype=np.float64)
    f = np.where(k < n // 2, k, k - n) * (f_s / n)
    return float(sideband) * f


def chirp_cycles(f_c, f, dm, k_dm=K_DM):
    """Phase of the dedispersion filter in cycles, and its reduction to [-1/2, 1/2].

    Integrating the group delay of Eq. dmdelay over frequency gives the ISM
    phase 2 pi K DM / (f_c + f).  Its expansion about f_c is
    K DM [1/f_c - f/f_c^2 + f^2/(f_c^2 (f_c + f))]; the constant and the linear
    (pure delay of the channel centre) terms are dropped as Sec. 2.1 drops them
    for the chirp, leaving u = K DM f^2 / (f_c^2 (f_c + f)) cycles.  Returns
    (u, r) with r = u - rint(u).
    """
    f = np.asarray(f, dtype=np.float64)
    u = (k_dm * dm) * (f * f) / (f_c * f_c * (f_c + f))
    r = u - np.rint(u)
    return u, r


def chirp(f_c, f_s, n, dm, sideband=1, k_dm=K_DM):
    """Coherent-dedispersion filter H[k] = exp(-2 pi i r_k) for one (channel, DM).

    The sign makes higher frequencies (which arrive first, Sec. 2.1) wait for
    the lower ones: the filter undoes the ISM (Sec. 2.3.2).
    """
    _, r = chirp_cycles(f_c, bin_offsets(n, f_s, sideband), dm, k_dm)
    return np.exp(-2j * np.pi * r)


def dedisperse_stream(x, h, fft_len, valid, lead, n_out=None):
    """Overlap-save convolution of x with the filter whose N-point DFT is h.

    x: [..., S] complex voltages (samples before 0 and from S on are zero).
    Block b takes input samples [b V - lead, b V - lead + N), is transformed
    with the unnormalised forward DFT, multiplied by h, inverse transformed
    (1/N), and its outputs lead .. lead+V-1 become y[b V .. b V + V - 1].
    """
    x = np.asarray(x)
    s = x.shape[-1]
    if n_out is None:
        n_out = s
    n = int(fft_len)
    nblocks = -(-n_out // valid)
    padded = np.zeros(x.shape[:-1] + (lead + nblocks * valid + n,), dtype=np.complex128)
    padded[..., lead:lead + s] = x
    y = np.zeros(x.shape[:-1] + (nblocks * valid,), dtype=np.complex128)
    for b in range(nblocks):
        win = padded[..., b * valid: b * valid + n]  # x[b V - lead + j]
        yb = np.fft.ifft(np.fft.fft(win, axis=-1) * h, axis=-1)
        y[..., b * valid:(b + 1) * valid] = yb[..., lead:lead + valid]
    return y[..., :n_out]


def correlate_dumps(y, dump_len):
    """Integrate-and-dump of the mixed products (Sec. 3.2 Eq. xpq; Sec. 5.1).

    y: [M, S] complex.  Returns V[m, i, j] = sum over n in [mL, (m+1)L) of
    y_i[n] conj(y_j[n]) for the floor(S/L) complete dumps.
    """
    m_ant, s = y.shape
    nd = s // dump_len
    # per dump m the L-sample block Y_m [M, L]; V[m] = Y_m Y_m^H (a matrix product)
    ym = y[:, :nd * dump_len].reshape(m_ant, nd, dump_len).transpose(1, 0, 2)
    return ym @ np.conj(ym).transpose(0, 2, 1)


def packed_index(i, j, m_ant):
    """Position of baseline (i, j), i <= j, in the packed upper triangle."""
    return i * m_ant - (i * (i - 1)) // 2 + (j - i)


def pack_upper(vfull):
    """[..., M, M] -> [..., M(M+1)/2] keeping i <= j in row-major order."""
    m_ant = vfull.shape[-1]
    iu, ju = np.triu_indices(m_ant)
    return vfull[..., iu, ju]


def _as_complex(volts):
    v = np.asarray(volts)
    if np.iscomplexobj(v):
        return v.astype(np.complex128)
    if v.dtype == np.int8:  # interleaved (re, im) int8, last axis 2*S
        return v[..., 0::2].astype(np.float64) + 1j * v[..., 1::2].astype(np.float64)
    raise TypeError("volts must be complex or interleaved int8")


def run_oracle(volts, chan_freqs, f_s, dm_lists, dump_len, blockings, sideband=1,
               k_dm=K_DM, quant=None, scales=None, chans=None, dm_index=None):
    """The whole pre-integrator stage for a set of channels.

    volts: [C, M, S] complex (or [C, M, 2S] interleaved int8).
    dm_lists[c]: trial DMs of channel c.  blockings[c]: dict with fft_len,
    valid and lead (the plan's blocking), or a list of such dicts, one per DM
    of the channel (each DM filtered with its own blocking).  quant: None, "e4m3" or "f16" to
    emulate the reduced-precision correlator inputs with per-channel scale
    scales[c]: the cross products V_ij (i != j) are those of the rounded
    voltages quantize(y s) / s^2, while the autocorrelations V_ii keep the
    unrounded voltages' power (reading: only the products between antennas
    take the narrow format; total power is formed at full precision).
    chans / dm_index restrict the work to some channels / DM indices.
    Returns {(c, d): V[dumps, M(M+1)/2]} complex128.
    """
    from .quant import quantize

    out = {}
    chans = range(len(chan_freqs)) if chans is None else chans
    for c in chans:
        x = _as_complex(volts[c])
        bl = blockings[c]
        dms = dm_lists[c]
        ds = range(len(dms)) if dm_index is None else dm_index
        for d in ds:
            b = bl[d] if isinstance(bl, (list, tuple)) else bl
            h = chirp(chan_freqs[c], f_s, b["fft_len"], dms[d], sideband, k_dm)
            y = dedisperse_stream(x, h, b["fft_len"], b["valid"], b["lead"])
            v = correlate_dumps(y, dump_len)
            if quant is not None:
                # cross products from the rounded inputs; the autocorrelations
                # (total power) stay those of the unrounded voltages
                s = float(scales[c])
                vq = correlate_dumps(quantize(y * s, quant), dump_len) / (s * s)
                idx = np.arange(v.shape[-1])
                vq[:, idx, idx] = v[:, idx, idx]
                v = vq
            out[(c, d)] = pack_upper(v)
    return out


def channel_delays(chan_freqs, dms, f_s, k_dm=K_DM, f_ref=None):
    """DM-delay bookkeeping from Eq. dmdelay (Sec. 2.1).

    delta[c, d] = K DM_d / f_c^2 seconds (delay of the channel centre behind
    infinite frequency) and shift[c, d] = rint(K DM_d (f_c^-2 - f_ref^-2) f_s)
    samples behind the reference frequency (default: highest channel centre).
    """
    fc = np.asarray(chan_freqs, dtype=np.float64)
    dm = np.asarray(dms, dtype=np.float64)
    if f_ref is None:
        f_ref = float(np.max(fc))
    inv = 1.0 / (fc * fc)
    delta = k_dm * dm[None, :] * inv[:, None]
    shift = np.rint(k_dm * dm[None, :] * (inv[:, None] - 1.0 / (f_ref * f_ref)) * f_s).astype(np.int64)
    return delta, shift


def dump_times(n_dumps, dump_len, f_s, first_dump=0, delay_s=0.0):
    """Time (s) of each dump, measured from the stream's first sample.

    Reading (the paper only names the integrate-and-dump cadence, Sec. 5.1):
    sample n is taken at n / f_s, and a dump stands at the mean time of the L
    samples it sums, (m L + (L - 1) / 2) / f_s.  Because the dedispersed
    voltages are index-aligned with the input, that is when the dump's signal
    reached the channel centre; subtracting delay_s = K DM / f_c^2 (the channel
    centre's delay behind infinite frequency, Eq. dmdelay) refers the dump to
    infinite frequency, the same time in every channel.
    """
    m = np.arange(first_dump, first_dump + n_dumps, dtype=np.float64)
    return (m * dump_len + 0.5 * (dump_len - 1)) / f_s - delay_s
