"""Host-side pieces of bench.py (no GPU): the one-GPU guard, the committed counter
records' validity against the kernel sources they were taken on, and the
provenance of the committed proposal weights."""
import json
import os
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""  # no JSON line


def test_counter_records_match_their_sources():
    """Every committed traffic record names the hash of the sources it was taken on;
    the records the bench line uses are current, and a record whose hash differs
    is ignored (traffic null)."""
    import bench
    for kernel, workload, sources in (("dedisperse", "c1", bench.DEDISP_SOURCES),
                                      ("correlate", "c1", bench.DEDISP_SOURCES),
                                      ("image", "chirp", bench.IMAGE_SOURCES),
                                      ("tree", "incoherent", bench.INCOHERENT_SOURCES),
                                      ("pre", "chimg", bench.CHIMG_SOURCES)):
        path = os.path.join(ROOT, "profiles", "traffic_%s_%s.json" % (kernel, workload))
        rec = json.load(open(path))
        assert rec["source_hash"] == bench.kernel_source_hash(sources), path
        assert bench.measured_traffic(kernel, workload, sources) == rec["bytes_per_launch"]
    # another source set hashes differently, so the record is not taken for it
    assert bench.measured_traffic("dedisperse", "c1", bench.IMAGE_SOURCES) is None
    assert bench.measured_traffic("nonexistent", "c1") is None


def test_dedisperse_record_is_consistent():
    """The dedispersion record's bytes per launch are its counters times the copy
    calibration, and its algorithmic bytes are the method's minimum per unit times
    the units of an average launch."""
    rec = json.load(open(os.path.join(ROOT, "profiles", "traffic_dedisperse_c1.json")))
    cal = rec["calibration"]
    got = (rec["fetch_kib_per_launch"] * cal["fetch"] + rec["write_kib_per_launch"] * cal["write"]) * 1024
    assert abs(got - rec["bytes_per_launch"]) <= 1e-6 * rec["bytes_per_launch"] + 2048
    assert rec["algorithmic_bytes_per_launch"] < rec["bytes_per_launch"]


def test_committed_weights_provenance():
    import bench
    path = os.path.join(ROOT, "paper_1109_3186_amd", "proposal_weights.npz")
    assert bench.weights_provenance(path) == "trained in fp16 on 100000 tiles"
    with np.load(path) as z:
        from paper_1109_3186_amd.binding import lib  # noqa: F401  (the library builds and loads on the CPU)
        import ctypes as ct
        n = ct.c_int64()
        lib().ddx_cnn_num_params(ct.byref(n))
        assert z["params"].shape == (n.value,)
        assert np.all(np.isfinite(z["params"]))
