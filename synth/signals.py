"""Voltage-stream generators (noise, int8 digitisation, dispersed pulses)."""

import math

import numpy as np

# Physical dispersion constant of the sky model, s Hz^2 cm^3 / pc.
K_DM_SKY = 4.148808e15
C_LIGHT = 299792458.0


def chan_freqs(f_lo, n_chan, f_s):
    """Centre sky frequency of each of n_chan contiguous channels of width f_s."""
    return f_lo + (np.arange(n_chan, dtype=np.float64) + 0.5) * f_s


def dm_grid(n, dm_max):
    """n trial DMs uniform on [0, dm_max), endpoint excluded: d * dm_max / n."""
    return np.arange(n, dtype=np.float64) * (dm_max / n)


def noise_complex(rng, shape, power=1.0):
    """Circular complex Gaussian noise with E|n|^2 = power."""
    s = math.sqrt(power / 2.0)
    return (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)) * s


def to_ci8(z):
    """Digitise complex values to interleaved int8 (RNE, clipped to +-127)."""
    z = np.asarray(z)
    out = np.empty(z.shape[:-1] + (2 * z.shape[-1],), dtype=np.int8)
    out[..., 0::2] = np.clip(np.rint(z.real), -127, 127).astype(np.int8)
    out[..., 1::2] = np.clip(np.rint(z.imag), -127, 127).astype(np.int8)
    return out


def antenna_positions(rng, m, radius_m):
    """m antennas uniform over a disk of the given radius (metres), [m, 2] (east, north)."""
    r = radius_m * np.sqrt(rng.random(m))
    th = 2.0 * np.pi * rng.random(m)
    return np.stack([r * np.cos(th), r * np.sin(th)], axis=-1)


def direction_grid(lmax, n, block=16):
    """n x n direction cosines (l, m) evenly over [-lmax, lmax]^2, [n * n, 2], listed
    in block x block tiles of neighbouring directions."""
    ax = np.linspace(-lmax, lmax, n)
    out = []
    for bi in range(0, n, block):
        for bj in range(0, n, block):
            for i in range(bi, min(n, bi + block)):
                for j in range(bj, min(n, bj + block)):
                    out.append((ax[i], ax[j]))
    return np.array(out, dtype=np.float64)


def _smear(f_c, f_s, dm, k_dm):
    hi, lo = f_c + 0.5 * f_s, f_c - 0.5 * f_s
    early = k_dm * dm * (1.0 / (f_c * f_c) - 1.0 / (hi * hi)) * f_s
    late = k_dm * dm * (1.0 / (lo * lo) - 1.0 / (f_c * f_c)) * f_s
    return early, late


def dispersed_segment(wave, f_c, f_s, dm, f_ref, delays=None, phases=None, k_dm=K_DM_SKY):
    """The dispersed pulse as received in one channel by each antenna.

    wave: [w] complex emitted waveform.  The pulse start reaches frequency
    f_ref at sample n0; this returns (offset, seg) with seg [M, Nseg] to be
    added to the stream from sample n0 + offset.  The sky model multiplies the
    spectrum by the cold-plasma response exp(2 pi i K DM / nu), nu = f_c + f
    (group delay K DM / nu^2, Eq. dmdelay), minus its constant phase; the
    channel-centre delay K DM (f_c^-2 - f_ref^-2) is split into a whole-sample
    shift and a fractional phase ramp.  Per antenna, either a geometric delay
    (seconds, applied at the full sky frequency) or a phase (radians) is added.
    """
    wave = np.asarray(wave, dtype=np.complex128)
    w = wave.shape[0]
    if delays is None and phases is None:
        phases = np.zeros(1)
    m_ant = len(delays) if delays is not None else len(phases)
    early, late = _smear(f_c, f_s, dm, k_dm)
    gmax = 0.0 if delays is None else float(np.max(np.abs(delays))) * f_s
    centre = k_dm * dm * (1.0 / (f_c * f_c) - 1.0 / (f_ref * f_ref)) * f_s
    ishift = int(math.floor(centre))
    frac = centre - ishift
    pad = int(math.ceil(early + gmax)) + 256
    span = pad + w + int(math.ceil(late + gmax + 1.0)) + 256
    nseg = 1 << int(math.ceil(math.log2(2 * span)))
    buf = np.zeros(nseg, dtype=np.complex128)
    buf[pad:pad + w] = wave
    spec = np.fft.fft(buf)
    f = np.fft.fftfreq(nseg, 1.0 / f_s)
    # K DM (1/nu - 1/f_c + f/f_c^2) written without the cancelling terms.
    cyc = k_dm * dm * (f / (f_c * f_c) - f / (f_c * (f_c + f))) - f * (frac / f_s)
    seg = np.empty((m_ant, nseg), dtype=np.complex128)
    for p in range(m_ant):
        c = cyc
        if delays is not None:
            c = cyc - (f_c + f) * delays[p]
        s = np.fft.ifft(spec * np.exp(2j * np.pi * np.mod(c, 1.0)))
        if phases is not None:
            s = s * np.exp(1j * phases[p])
        seg[p] = s
    return ishift - pad, seg


def dispersed_segment_device(wave, f_c, f_s, dm, f_ref, delays, device, k_dm=K_DM_SKY):
    """dispersed_segment with per-antenna geometric delays, evaluated on a torch
    device in float64 (the same phases; the inverse FFTs of all antennas at once).
    Returns (offset, seg) with seg a complex128 tensor [M, Nseg]."""
    import torch

    wave = np.asarray(wave, dtype=np.complex128)
    w = wave.shape[0]
    early, late = _smear(f_c, f_s, dm, k_dm)
    gmax = float(np.max(np.abs(delays))) * f_s
    centre = k_dm * dm * (1.0 / (f_c * f_c) - 1.0 / (f_ref * f_ref)) * f_s
    ishift = int(math.floor(centre))
    frac = centre - ishift
    pad = int(math.ceil(early + gmax)) + 256
    span = pad + w + int(math.ceil(late + gmax + 1.0)) + 256
    nseg = 1 << int(math.ceil(math.log2(2 * span)))
    buf = np.zeros(nseg, dtype=np.complex128)
    buf[pad:pad + w] = wave
    spec = torch.from_numpy(np.fft.fft(buf)).to(device)
    f = np.fft.fftfreq(nseg, 1.0 / f_s)
    cyc = k_dm * dm * (f / (f_c * f_c) - f / (f_c * (f_c + f))) - f * (frac / f_s)
    c = torch.from_numpy(cyc).to(device)[None, :] - torch.from_numpy(f_c + f).to(device)[None, :] * \
        torch.from_numpy(np.asarray(delays, np.float64)).to(device)[:, None]
    ph = torch.remainder(c, 1.0) * (2.0 * math.pi)
    seg = torch.fft.ifft(spec[None, :] * torch.polar(torch.ones_like(ph), ph), dim=-1)
    return ishift - pad, seg


def inject_pulse(stream, f_c, f_s, dm, n0, wave, f_ref, delays=None, phases=None, k_dm=K_DM_SKY):
    """Add the dispersed pulse to stream [M, S] (complex, in place); returns the stream."""
    off, seg = dispersed_segment(wave, f_c, f_s, dm, f_ref, delays, phases, k_dm)
    s = stream.shape[-1]
    a = n0 + off
    lo, hi = max(a, 0), min(a + seg.shape[-1], s)
    if hi > lo:
        stream[:, lo:hi] += seg[:, lo - a:hi - a]
    return stream


def pulse_wave(rng, width, snr, noise_power):
    """Boxcar of complex Gaussian source noise with matched-filter S/N ``snr``."""
    amp2 = snr * noise_power / math.sqrt(width)
    return noise_complex(rng, (width,), amp2)


def make_c0(seed=1109, with_pulse=True):
    """8 antennas, one 1 MHz channel at 1.4 GHz, 65536 unit-variance samples,
    one pulse at DM 50 (100 us, S/N 20, random per-antenna phase); 16 trial
    DMs uniform over 0-100; FFT 4096; dumps of 64 samples."""
    rng = np.random.Generator(np.random.PCG64(seed))
    m_ant, s, f_s = 8, 65536, 1.0e6
    fc = np.array([1.4e9])
    x = noise_complex(rng, (1, m_ant, s))
    pulse = {"dm": 50.0, "width": 100, "snr": 20.0, "n0": 30000}
    if with_pulse:
        wave = pulse_wave(rng, pulse["width"], pulse["snr"], 1.0)
        phases = 2.0 * np.pi * rng.random(m_ant)
        inject_pulse(x[0], fc[0], f_s, pulse["dm"], pulse["n0"], wave, f_ref=fc[0], phases=phases)
        pulse["phases"] = phases
    return {
        "volts": x.astype(np.complex64), "chan_freqs": fc, "f_s": f_s,
        "dm_lists": [dm_grid(16, 100.0)], "dump_len": 64, "fft_len": 4096,
        "pulses": [pulse] if with_pulse else [],
    }


def make_small(seed, m_ant, n_chan, s, f_lo, f_s, n_dm, dm_max, dump_len, fft_len=0,
               ci8=False, sigma=16.0, n_pulses=1, snr=20.0, width=100, radius_m=3000.0):
    """A small multi-channel stream with the statistics of the larger workloads."""
    rng = np.random.Generator(np.random.PCG64(seed))
    fc = chan_freqs(f_lo, n_chan, f_s)
    power = 2.0 * sigma * sigma if ci8 else 1.0
    x = noise_complex(rng, (n_chan, m_ant, s), power)
    pos = antenna_positions(rng, m_ant, radius_m)
    f_ref = float(fc[-1])
    pulses = []
    for _ in range(n_pulses):
        dm = float(rng.uniform(0.0, dm_max))
        l, mm = rng.uniform(-0.02, 0.02, 2)
        delays = (pos[:, 0] * l + pos[:, 1] * mm) / C_LIGHT
        sweep = K_DM_SKY * dm * (1.0 / fc[0] ** 2 - 1.0 / f_ref ** 2) * f_s
        e0, l0 = _smear(fc[0], f_s, dm, K_DM_SKY)
        lo = int(e0) + 64
        hi = s - int(sweep + l0) - width - 64
        n0 = int(rng.integers(lo, max(hi, lo + 1)))
        waves = [pulse_wave(rng, width, snr, power) for _ in range(n_chan)]
        for c in range(n_chan):
            inject_pulse(x[c], fc[c], f_s, dm, n0, waves[c], f_ref, delays=delays)
        pulses.append({"dm": dm, "n0": n0, "width": width, "snr": snr, "lm": (l, mm)})
    volts = to_ci8(x) if ci8 else x.astype(np.complex64)
    return {
        "volts": volts, "chan_freqs": fc, "f_s": f_s,
        "dm_lists": [dm_grid(n_dm, dm_max) for _ in range(n_chan)],
        "dump_len": dump_len, "fft_len": fft_len, "pulses": pulses, "positions": pos,
    }


def c1_params():
    """36 antennas in a 3 km-radius disk, 64 x 1 MHz channels over 1.2-1.264 GHz,
    2^20 complex-int8 samples per channel (sigma 16), 256 trial DMs over 0-2000,
    1 ms dumps, 10 pulses (100 us, S/N 20) at random DM, time and position."""
    return {"m_ant": 36, "n_chan": 64, "samples": 1 << 20, "f_lo": 1.2e9, "f_s": 1.0e6,
            "n_dm": 256, "dm_max": 2000.0, "dump_len": 1000, "sigma": 16.0,
            "n_pulses": 10, "snr": 20.0, "width": 100, "radius_m": 3000.0, "seed": 1110}


def c3_params():
    """256 antennas in a 5 km-diameter disk, 32 x 1 MHz channels over
    0.7-0.732 GHz, 2^18 complex-int8 samples, per-channel DM grids of
    512 + round(1024 c / 31) trials over 0-3000, 1 ms dumps."""
    return {"m_ant": 256, "n_chan": 32, "samples": 1 << 18, "f_lo": 0.7e9, "f_s": 1.0e6,
            "n_dm": [512 + int(round(1024 * c / 31)) for c in range(32)], "dm_max": 3000.0,
            "dump_len": 1000, "sigma": 16.0, "n_pulses": 10, "snr": 20.0, "width": 100,
            "radius_m": 2500.0, "seed": 1112}


def pulse_channels_device(pl, fc, f_s, f_ref, pos, noise_power, device, k_dm=K_DM_SKY, chan_ids=None):
    """One pulse as received in every channel of fc by every antenna, on a torch
    device in float64: the model of dispersed_segment_device (cold-plasma response
    minus its constant phase, whole-sample shift plus fractional ramp, geometric
    delays at the full sky frequency) with one segment length for all channels.
    The waveform of row c comes from PCG64(wave_seed + chan_ids[c]) (chan_ids:
    the channels' indices in their stream, default 0, 1, ...).
    Returns (offsets [C] int, seg complex128 tensor [C, M, Nseg]): segment c is
    added to the stream of channel c from sample n0 + offsets[c]."""
    import torch

    fc = np.asarray(fc, dtype=np.float64)
    w, dm = pl["width"], pl["dm"]
    delays = (pos[:, 0] * pl["lm"][0] + pos[:, 1] * pl["lm"][1]) / C_LIGHT
    gmax = float(np.max(np.abs(delays))) * f_s
    early, late = _smear(fc, f_s, dm, k_dm)
    centre = k_dm * dm * (1.0 / (fc * fc) - 1.0 / (f_ref * f_ref)) * f_s
    ishift = np.floor(centre).astype(np.int64)
    frac = centre - ishift
    pad = np.ceil(early + gmax).astype(np.int64) + 256
    span = pad + w + np.ceil(late + gmax + 1.0).astype(np.int64) + 256
    nseg = 1 << int(math.ceil(math.log2(2 * int(span.max()))))
    buf = np.zeros((len(fc), nseg), dtype=np.complex128)
    ids = range(len(fc)) if chan_ids is None else chan_ids
    for c, cid in enumerate(ids):
        wrng = np.random.Generator(np.random.PCG64(pl["wave_seed"] + int(cid)))
        buf[c, pad[c]:pad[c] + w] = pulse_wave(wrng, w, pl["snr"], noise_power)
    spec = torch.fft.fft(torch.from_numpy(buf).to(device), dim=-1)
    f = torch.from_numpy(np.fft.fftfreq(nseg, 1.0 / f_s)).to(device)[None, :]
    fct = torch.from_numpy(fc).to(device)[:, None]
    # K DM (1/nu - 1/f_c + f/f_c^2) written without the cancelling terms
    cyc = k_dm * dm * (f / (fct * fct) - f / (fct * (fct + f))) - f * torch.from_numpy(frac / f_s).to(device)[:, None]
    ph = cyc[:, None, :] - (fct + f)[:, None, :] * torch.from_numpy(np.asarray(delays, np.float64)).to(device)[None, :, None]
    ph = torch.remainder(ph, 1.0) * (2.0 * math.pi)
    seg = torch.fft.ifft(spec[:, None, :] * torch.polar(torch.ones_like(ph), ph), dim=-1)
    return ishift - pad, seg


def make_stream_device(p, device, chans=None):
    """Build the complex-int8 stream [C, M, 2S] of workload ``p`` on a torch device.

    Noise comes from torch's seeded generator (one seed per channel), pulses
    from PCG64 on the host; the sum is rounded half-to-even and clipped.
    Returns (tensor, pulses, chan_freqs, positions).
    """
    import torch

    rng = np.random.Generator(np.random.PCG64(p["seed"]))
    m_ant, n_chan, s, f_s = p["m_ant"], p["n_chan"], p["samples"], p["f_s"]
    fc = chan_freqs(p["f_lo"], n_chan, f_s)
    pos = antenna_positions(rng, m_ant, p["radius_m"])
    f_ref = float(fc[-1])
    power = 2.0 * p["sigma"] ** 2
    pulses = []
    for _ in range(p["n_pulses"]):
        dm = float(rng.uniform(0.0, p["dm_max"]))
        l, mm = rng.uniform(-0.02, 0.02, 2)
        sweep = K_DM_SKY * dm * (1.0 / fc[0] ** 2 - 1.0 / f_ref ** 2) * f_s
        e0, l0 = _smear(fc[0], f_s, dm, K_DM_SKY)
        lo = int(e0) + 64
        hi = s - int(sweep + l0) - p["width"] - 64
        n0 = int(rng.integers(lo, max(hi, lo + 1)))
        pulses.append({"dm": dm, "n0": n0, "width": p["width"], "snr": p["snr"], "lm": (l, mm),
                       "wave_seed": int(rng.integers(0, 2 ** 31))})
    chans = list(range(n_chan) if chans is None else chans)
    out = torch.empty((len(chans), m_ant, 2 * s), dtype=torch.int8, device=device)
    re = torch.empty((len(chans), m_ant, s), dtype=torch.float32, device=device)
    im = torch.empty_like(re)
    for ci, c in enumerate(chans):
        g = torch.Generator(device=device)
        g.manual_seed(p["seed"] * 1000 + int(c))
        re[ci] = torch.randn((m_ant, s), generator=g, device=device, dtype=torch.float32) * p["sigma"]
        im[ci] = torch.randn((m_ant, s), generator=g, device=device, dtype=torch.float32) * p["sigma"]
    # channels in groups small enough that one group's segments stay near 1 GiB
    group = max(1, 1024 // m_ant)
    for pl in pulses:
        for g0 in range(0, len(chans), group):
            sub = chans[g0:g0 + group]
            off, seg = pulse_channels_device(dict(pl, snr=p["snr"]), fc[sub], f_s, f_ref, pos, power, device,
                                             chan_ids=sub)
            for k in range(len(sub)):
                ci = g0 + k
                a = pl["n0"] + int(off[k])
                lo, hi = max(a, 0), min(a + seg.shape[-1], s)
                if hi > lo:
                    part = seg[k, :, lo - a:hi - a]
                    re[ci, :, lo:hi] += part.real.to(torch.float32)
                    im[ci, :, lo:hi] += part.imag.to(torch.float32)
            del seg
    out[..., 0::2] = torch.clamp(torch.round(re), -127, 127).to(torch.int8)
    out[..., 1::2] = torch.clamp(torch.round(im), -127, 127).to(torch.int8)
    del re, im
    return out, pulses, fc, pos
