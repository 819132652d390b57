"""GPU test of the autotuner: it measures, caches, reuses the cache, and the
plan it configures stays within parity of the FP64 oracle."""
import json

import numpy as np
import pytest

import synth
from gpu_helpers import compare_with_oracle, run_gpu, say

pytestmark = pytest.mark.gpu


def test_tune_cache_and_parity(gpu, tmp_path):
    from paper_1109_3186_amd import autotune
    cfg = synth.make_small(seed=70, m_ant=4, n_chan=3, s=60000, f_lo=1.2e9, f_s=1e6, n_dm=6, dm_max=400.0,
                           dump_len=100, ci8=True, n_pulses=1)
    cache = str(tmp_path / "tune.json")
    r1 = autotune.tune(4, cfg["chan_freqs"], 1e6, 100, cfg["dm_lists"], in_dtype="ci8", max_block=60000,
                       cache=cache, dm_sample=4, log=say)
    assert r1["source"] == "measured"
    assert len(r1["fft_len"]) == 3 and all(n in (r1["auto_fft_len"][c] // 2, r1["auto_fft_len"][c],
                                                 2 * r1["auto_fft_len"][c], 4 * r1["auto_fft_len"][c])
                                           for c, n in enumerate(r1["fft_len"]))
    db = json.load(open(cache))
    assert len(db) == 1
    r2 = autotune.tune(4, cfg["chan_freqs"], 1e6, 100, cfg["dm_lists"], in_dtype="ci8", max_block=60000,
                       cache=cache, dm_sample=4)
    assert r2["source"] == "cache" and r2["fft_len"] == r1["fft_len"]
    vis, lay = run_gpu(cfg, in_dtype="ci8", fft_len=r1["fft_len"], wave_units=r1["wave_units"],
                       dm_group=r1["dm_group"])
    assert list(lay["fft_len"]) == r1["fft_len"]
    err = compare_with_oracle(cfg, vis, lay)
    say("tuned lengths %s wave %d group %d: max normalised error %.3e" % (
        r1["fft_len"], r1["wave_units"], r1["dm_group"], err))
    assert err <= 1e-5
