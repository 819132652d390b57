"""GPU test of the autotuner: it measures, caches, reuses the cache, and the
plan it configures stays within parity of the FP64 oracle."""
import json

import numpy as np
import pytest

import synth
from gpu_helpers import compare_with_oracle, run_gpu, say

pytestmark = pytest.mark.gpu


def test_tune_cache_and_parity(gpu, tmp_path):
    """The tuner measures a cost table (positive and finite; on a workload this small
    launch overheads dominate it), caches it with the schedule, reuses the cache,
    and a plan built from it cuts its classes by that table (the host rule with the
    same table agrees) and stays within parity."""
    from paper_1109_3186_amd import autotune, plan_blocking
    cfg = synth.make_small(seed=70, m_ant=4, n_chan=3, s=60000, f_lo=1.2e9, f_s=1e6, n_dm=6, dm_max=400.0,
                           dump_len=100, ci8=True, n_pulses=1)
    cfg["dm_lists"][0] = np.linspace(0.0, 1500.0, 40)
    cache = str(tmp_path / "tune.json")
    r1 = autotune.tune(4, cfg["chan_freqs"], 1e6, 100, cfg["dm_lists"], in_dtype="ci8", max_block=60000,
                       cache=cache, dm_sample=4, log=say)
    assert r1["source"] == "measured"
    cost = np.array(r1["cost_ps"])
    say("cost table (ps per point, N 2^8 .. 2^18):", np.round(cost, 2).tolist())
    assert cost.shape == (2, 11) and np.all(cost > 0) and np.all(np.isfinite(cost))
    db = json.load(open(cache))
    assert len(db) == 1
    r2 = autotune.tune(4, cfg["chan_freqs"], 1e6, 100, cfg["dm_lists"], in_dtype="ci8", max_block=60000,
                       cache=cache, dm_sample=4)
    assert r2["source"] == "cache" and r2["cost_ps"] == r1["cost_ps"]
    kw = autotune.plan_kwargs(r1)
    vis, lay = run_gpu(cfg, in_dtype="ci8", **kw)
    n, v, l, k = plan_blocking(cfg["chan_freqs"][:1], 1e6, 100, cfg["dm_lists"][0], cost_ps=kw["cost_ps"])
    off = lay["dm_offset"]
    assert np.array_equal(lay["dm_fft_len"][off[0]:off[1]], n) and np.array_equal(lay["dm_valid"][off[0]:off[1]], v)
    err = compare_with_oracle(cfg, vis, lay)
    say("tuned: %d classes, wave %d group %d: max normalised error %.3e" % (
        lay["n_classes"], r1["wave_units"], r1["dm_group"], err))
    assert err <= 1e-5
