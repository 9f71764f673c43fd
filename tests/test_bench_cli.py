"""Host logic of the benchmark's command line (CPU only): the path runs on one
GPU, so a request for more exits with a message before touching a device."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], cwd=ROOT,
                       capture_output=True, text=True, timeout=300)
    assert p.returncode == 2, p.stderr[-2000:]
    line = json.loads(p.stdout.strip().splitlines()[-1])
    assert "one GPU" in line["error"]
