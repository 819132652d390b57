"""Checks of the seeded input generators (host side)."""
import numpy as np

import synth


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def test_device_segment_matches_host_segment():
    """The torch form of the dispersed pulse (used for device-generated streams) gives
    the same samples as the NumPy form (here on the CPU)."""
    rng = _rng(91)
    wave = synth.pulse_wave(rng, 100, 20.0, 512.0)
    delays = rng.uniform(-3e-6, 3e-6, 5)
    o1, s1 = synth.signals.dispersed_segment(wave, 0.7005e9, 1e6, 300.0, 0.7315e9, delays=delays)
    o2, s2 = synth.signals.dispersed_segment_device(wave, 0.7005e9, 1e6, 300.0, 0.7315e9, delays, "cpu")
    assert o1 == o2
    assert np.max(np.abs(s2.numpy() - s1)) <= 1e-9 * np.max(np.abs(s1))


def test_all_channel_pulse_matches_per_channel_segments():
    """The batched form (one segment length for every channel) places the same
    dispersed pulse as the per-channel form, up to the chirp response's far tails,
    which wrap differently in the longer segment."""
    import math
    rng = _rng(92)
    pos = synth.antenna_positions(rng, 4, 3000.0)
    fc = synth.chan_freqs(1.2e9, 3, 1e6)
    pl = {"dm": 900.0, "width": 100, "snr": 20.0, "lm": (0.01, -0.015), "wave_seed": 77}
    off, seg = synth.signals.pulse_channels_device(pl, fc, 1e6, float(fc[-1]), pos, 512.0, "cpu")
    seg = seg.numpy()
    delays = (pos[:, 0] * pl["lm"][0] + pos[:, 1] * pl["lm"][1]) / synth.signals.C_LIGHT
    for c in range(3):
        wave = synth.pulse_wave(np.random.Generator(np.random.PCG64(77 + c)), 100, 20.0, 512.0)
        o1, s1 = synth.signals.dispersed_segment(wave, fc[c], 1e6, 900.0, float(fc[-1]), delays=delays)
        n = 1 << 17
        a = np.zeros((4, n), complex)
        b = np.zeros((4, n), complex)
        base = 40000
        a[:, base + o1:base + o1 + s1.shape[1]] = s1
        b[:, base + int(off[c]):base + int(off[c]) + seg.shape[2]] = seg[c]
        peak = np.abs(a).max()
        assert np.max(np.abs(a - b)) <= 2e-3 * peak, (c, np.max(np.abs(a - b)) / peak)
        assert math.isclose(np.sum(np.abs(a) ** 2), np.sum(np.abs(b) ** 2), rel_tol=1e-3)
