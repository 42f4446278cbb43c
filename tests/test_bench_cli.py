"""bench.py command line (CPU only): one GPU only, and the JSON contract of the
refusal line."""

import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert line["n_gpus"] == 2 and "one GPU" in line["error"]


def test_profiled_traffic_follows_the_sources():
    """The roofline traffic figure is reported only for a profiled workload
    whose kernel sources still hash to the profiled ones."""
    sys.path.insert(0, ROOT)
    import bench
    t = bench.profiled_traffic("batched4500")
    # plausible: at least the 12 bytes of coordinates per source point, at
    # most three times the 3.88 GB of algorithmic bytes per round
    assert t is None or 12 * 101_596_832 < t < 3 * 3.88e9
    assert bench.profiled_traffic("batched4500", 1536) is None
    assert bench.profiled_traffic("batched4500", None, "interleaved") is None
    assert bench.profiled_traffic("no_such_workload") is None


def test_single_process_oracle_rate_and_host_model():
    """The baseline's one-process oracle rate runs in-process on a bounded
    sample and the host's CPU model is named."""
    import bench
    from synth import make_tiny_workload
    w = make_tiny_workload(seed=3, n_src=[300, 200], n_tgt=[400, 300], resolution=0.5,
                           n_factors=2, half=4.0, height=2.0)
    rate, n = bench.cpu_single_process(w, seconds=0.2)
    assert n >= 1 and rate >= 0.0
    assert bench.host_cpu_model()
