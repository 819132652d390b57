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
