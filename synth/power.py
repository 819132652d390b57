"""Beam power at the detected-power level, for DM-time training tiles.

A tile of a real stream sums |x|^2 over antennas and samples; generating 10^5
streams of voltages for training would move petabytes, so training tiles are
made from beam power drawn at fine-bin resolution with the same statistics:

* noise: each fine bin of F samples sums M F values |x|^2 of circular complex
  Gaussian noise with E|x|^2 = 2 sigma^2, a Gamma(M F, 2 sigma^2) variable, drawn
  here from its normal approximation (M F = 1152 for the 36-antenna workload);
* a pulse adds its energy M w a^2 (a^2 = SNR 2 sigma^2 / sqrt(w), the same
  amplitude rule as the voltage generator) spread uniformly over its sweep
  through the channel: from the arrival of the channel's top edge to that of its
  bottom edge plus the width, with the channel-centre delay of Eq. dmdelay.

Labels: 1 for every trial within one trial spacing of an injected DM.
The project's tile kernel turns this power into tiles exactly as it turns the
power of voltage streams into tiles.
"""

import math

import numpy as np

from .signals import K_DM_SKY, _smear, chan_freqs


def sample_pulses(rng, n_samples, fc, f_s, dm_max, snr_range, width, n_pulses):
    """Random pulses (DM, arrival at the highest channel, S/N) whose sweep fits in the stream."""
    f_ref = float(fc[-1])
    out = []
    for _ in range(n_pulses):
        dm = float(rng.uniform(0.0, dm_max))
        snr = float(rng.uniform(*snr_range))
        sweep = K_DM_SKY * dm * (1.0 / fc[0] ** 2 - 1.0 / f_ref ** 2) * f_s
        e0, l0 = _smear(fc[0], f_s, dm, K_DM_SKY)
        lo = int(e0) + 64
        hi = n_samples - int(sweep + l0) - width - 64
        n0 = int(rng.integers(lo, max(hi, lo + 1)))
        out.append({"dm": dm, "n0": n0, "snr": snr, "width": width})
    return out


def power_batch(p, n_tiles, fine, rng, gen, device, pulse_frac=0.5, snr_range=(5.0, 50.0), max_pulses=3,
                pulses_given=None):
    """Fine-bin beam power [n_tiles, C, U] (torch float32 on `device`), DM labels
    [n_tiles, D] and the pulse lists, for workload parameters p (see c1_params).
    pulses_given: optional list (one per tile) of pulse lists (dm, n0, snr, width)
    to inject instead of random ones."""
    import torch

    m_ant, n_chan, s, f_s = p["m_ant"], p["n_chan"], p["samples"], p["f_s"]
    units = s // fine
    fc = chan_freqs(p["f_lo"], n_chan, f_s)
    f_ref = float(fc[-1])
    var = 2.0 * p["sigma"] ** 2                       # E|x|^2 per sample
    k = m_ant * fine
    mean, sd = k * var, math.sqrt(k) * var          # Gamma(k, var) moments
    power = torch.randn((n_tiles, n_chan, units), generator=gen, device=device, dtype=torch.float32) * sd + mean
    dstep = p["dm_max"] / p["n_dm"]
    labels = np.zeros((n_tiles, p["n_dm"]), dtype=np.float32)
    grid = torch.arange(units + 1, device=device, dtype=torch.float64)
    pulses = []
    for t in range(n_tiles):
        if pulses_given is not None:
            pl = pulses_given[t]
        else:
            npul = 0 if rng.random() < (1.0 - pulse_frac) else int(rng.integers(1, max_pulses + 1))
            pl = sample_pulses(rng, s, fc, f_s, p["dm_max"], snr_range, p["width"], npul)
        pulses.append(pl)
        for q in pl:
            energy = m_ant * math.sqrt(q["width"]) * q["snr"] * var
            shift = K_DM_SKY * q["dm"] * (1.0 / fc ** 2 - 1.0 / f_ref ** 2) * f_s
            early, late = _smear(fc, f_s, q["dm"], K_DM_SKY)
            s0 = q["n0"] + shift - early
            s1 = q["n0"] + shift + late + q["width"]
            u0 = torch.tensor(s0 / fine, device=device)[:, None]
            u1 = torch.tensor(s1 / fine, device=device)[:, None]
            dens = torch.tensor(energy / (s1 - s0) * fine, device=device)[:, None]
            ramp = dens * torch.clamp(torch.minimum(grid[None, :], u1) - u0, min=0.0)
            power[t] += (ramp[:, 1:] - ramp[:, :-1]).to(torch.float32)
            d0 = q["dm"] / dstep
            lo, hi = int(math.ceil(d0 - 1.0)), int(math.floor(d0 + 1.0))
            labels[t, max(lo, 0):min(hi, p["n_dm"] - 1) + 1] = 1.0
    return power, torch.from_numpy(labels).to(device), pulses
