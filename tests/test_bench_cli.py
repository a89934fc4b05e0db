"""Host-side checks of bench.py's command line (no GPU): more than one GPU is
refused with a JSON message, and every workload name parses."""

import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in line["error"]


def test_workload_names_parse():
    sys.path.insert(0, ROOT)
    import bench

    old = sys.argv
    try:
        for w in ("dense_large", "batched", "hetero", "sets", "silk", "refine", "quantile"):
            sys.argv = ["bench.py", "--workload", w, "--steps", "3", "--warmup", "1"]
            a = bench.parse()
            assert a.workload == w and a.steps == 3 and a.warmup == 1 and a.gpus == 1 and a.pipeline == 0
    finally:
        sys.argv = old
