"""bench.py's command line on the CPU: it rejects more than one GPU with a message before touching
a device, and its helpers (percentiles, algorithmic flop counts, the traffic record lookup) behave."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_percentile_and_flop_helpers():
    import bench
    from paper_2407_13950_amd import workloads as WL
    assert bench.percentile([3.0, 1.0, 2.0], 50) == 2.0
    assert bench.percentile([1.0, 2.0], 99) == pytest.approx(1.99)
    w = WL.c3()
    f_fwd, f_bwd = bench.algorithmic_flops(w, 4)
    # per entry-step: forward 122 flops, backward 292 (q = 4, L = 4, four half sweeps)
    entry_steps = w.N * w.E * w.n_steps
    assert f_fwd == pytest.approx(122 * entry_steps) and f_bwd == pytest.approx(292 * entry_steps)


def test_traffic_record_matches_only_its_kernel_and_source(tmp_path, monkeypatch):
    import bench
    rec = json.load(open(os.path.join(ROOT, "profiles", "traffic_k_backward_q4L4.json")))
    got = bench.measured_traffic(rec["kernel"])
    import hashlib
    h = hashlib.sha256()    # the kernels' sources and the build flags, in this order
    for rel in (("csrc", "qoc_kernels.hip"), ("csrc", "qoc_ilp_unit.hip"), ("build.py",)):
        h.update(open(os.path.join(ROOT, "paper_2407_13950_amd", *rel), "rb").read())
    sha = h.hexdigest()
    assert (got == rec["bytes_per_launch"]) == (sha == rec["source_sha256"])
    assert bench.measured_traffic("k_backward_x3<float, 4, 4, 3, false>") is None
