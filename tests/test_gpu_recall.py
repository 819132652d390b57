"""Voltage-level recall of the learned proposal over 100 streams of the 36-antenna
workload's shape (1000 injected pulses at S/N 20): the proposal alone keeps at
least 99 % of the pulses the full sweep can recover, and the power-model tiles the
network was trained on match the voltage-generated tiles of the same pulses."""
import os

import pytest

from gpu_helpers import say

pytestmark = pytest.mark.gpu

WEIGHTS = os.path.join(os.path.dirname(os.path.dirname(__file__)), "paper_1109_3186_amd", "proposal_weights.npz")


@pytest.mark.skipif(not os.path.exists(WEIGHTS), reason="no trained weights")
def test_recall_over_1000_pulses(gpu):
    import bench
    rec = bench.recall_study(gpu, n_streams=100)
    tv = rec["tile_validation"]
    say("recall %d/%d (%.4f; of sweep-recoverable %.4f), fallbacks %d, judged misses %s; tiles %s" % (
        rec["kept"], rec["pulses"], rec["recall"], rec["recall_of_sweep_recoverable"], rec["fallbacks"],
        rec["misses_judged_by_full_sweep"], tv))
    assert rec["pulses"] >= 1000
    assert rec["recall_of_sweep_recoverable"] >= 0.99
    # the shortcut reproduces the voltage tiles: pulse peaks within 15 % at the median,
    # noise spread within 10 %
    assert 0.85 <= tv["peak_ratio_median"] <= 1.15
    assert abs(tv["noise_sd_voltage"] / tv["noise_sd_power_model"] - 1.0) <= 0.10
