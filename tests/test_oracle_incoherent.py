"""Pins of the incoherent-dedispersion oracle (oracle/incoherent.py): the tree
method against brute force with the tree's own delays (exact on integer data),
the tree's sweeps against straight lines (endpoints exact, slope monotone, a
deviation that grows only logarithmically), impulses laid along a sweep or along
the dispersion law summing to the channel count, the DM delays' ordering and
rounding, and the power beam against a direct loop."""
import math

import numpy as np
import pytest

from oracle import incoherent as inc


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


@pytest.mark.parametrize("C,T", [(1, 7), (2, 9), (8, 40), (32, 70), (16, 3), (64, 20)])
def test_tree_equals_brute_force_with_its_delays(C, T):
    """Also with fewer samples than the largest sweep shift (those reads are zero)."""
    p = _rng(C).integers(0, 100, (C, T)).astype(np.float64)
    out = inc.tree(p)
    delays = np.array([inc.tree_delays(C, j) for j in range(C)]).T    # [C][sweeps]
    ref = inc.brute_force(p, delays, T)
    assert np.array_equal(out, ref)


@pytest.mark.parametrize("C", [2, 4, 16, 64, 256, 1024])
def test_tree_sweeps_are_near_straight_lines(C):
    """Sweep j delays channel 0 by 0 and the last by j, never decreasing; its
    largest distance from the line j c / (C - 1) is at most log2(C) / 6 samples."""
    for j in range(C):
        d = np.array(inc.tree_delays(C, j))
        assert d[0] == 0 and d[-1] == j and np.all(np.diff(d) >= 0)
        lin = j * np.arange(C) / (C - 1)
        assert np.max(np.abs(d - lin)) <= math.log2(C) / 6 + 1e-12


def test_tree_sweep_zero_is_the_channel_sum_and_impulses_add_up():
    C, T = 16, 60
    p = _rng(3).random((C, T))
    assert np.allclose(inc.tree(p)[0], p.sum(axis=0), rtol=0, atol=1e-12)
    for j0 in (0, 5, 15):
        q = np.zeros((C, T))
        for c, dc in enumerate(inc.tree_delays(C, j0)):
            q[c, 20 + dc] = 1.0
        out = inc.tree(q)
        assert out[j0, 20] == C and out.max() == C


def test_dm_delays_follow_the_dispersion_law():
    f = 1.2e9 + 1e6 * np.arange(8)[::-1]           # channel 0 highest
    dl = inc.dm_delays(f, 1e-3, [0.0, 500.0, 2000.0])
    assert np.all(dl[:, 0] == 0) and np.all(dl[0] == 0)
    assert np.all(np.diff(dl[:, 2]) >= 0)           # lower frequency, later
    # DM 2000 between 1.2 and 1.207 GHz: K DM (f_lo^-2 - f_hi^-2) = 66.6 ms
    sec = 4.148808e15 * 2000.0 * (1 / 1.2e9 ** 2 - 1 / 1.207e9 ** 2)
    assert dl[7, 2] == round(sec / 1e-3) == 67


def test_brute_force_recovers_a_dispersed_impulse():
    f = 1.2e9 + 1e6 * np.arange(32)[::-1]
    dms = np.linspace(0, 1000, 17)
    dl = inc.dm_delays(f, 1e-4, dms)
    T = int(dl.max()) + 200
    p = np.zeros((32, T))
    d0, t0 = 11, 150
    p[np.arange(32), t0 + dl[:, d0]] = 1.0
    out = inc.brute_force(p, dl, 200)
    assert out[d0, t0] == 32 and out.max() == 32
    assert np.allclose(inc.brute_force(p, np.zeros_like(dl), 200)[0], p[:, :200].sum(axis=0))


def test_power_beam_is_the_detected_sum():
    v = _rng(5).normal(size=(3, 4, 50)) + 1j * _rng(6).normal(size=(3, 4, 50))
    p = inc.power_beam(v, 8)
    assert p.shape == (3, 6)
    for c in range(3):
        for t in range(6):
            ref = sum(abs(v[c, a, n]) ** 2 for a in range(4) for n in range(8 * t, 8 * t + 8))
            assert abs(p[c, t] - ref) < 1e-10


def test_brute_force_is_the_plain_sum_for_any_delays():
    """Brute force on tiny inputs against the per-element definition, with delays
    before the first sample, past the last and spread widely."""
    rng = _rng(77)
    C, T, D = 5, 23, 9
    p = rng.random((C, T))
    dl = rng.integers(-30, 30, (C, D))
    for n_out in (1, 17, 40):
        ref = np.zeros((D, n_out))
        for d in range(D):
            for t in range(n_out):
                for c in range(C):
                    s = t + dl[c, d]
                    if 0 <= s < T:
                        ref[d, t] += p[c, s]
        assert np.allclose(inc.brute_force(p, dl, n_out), ref, rtol=0, atol=1e-12)
