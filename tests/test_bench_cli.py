"""bench.py's command-line contract that needs no GPU: more than one GPU is
refused with a message (the implementation runs on one GPU), and the rocprofv3
summarizer runs on the host."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert p.returncode == 2
    out = json.loads(p.stdout.strip().splitlines()[-1])
    assert out["n_gpus"] == 2 and "one GPU" in out["error"]


def test_summarize_without_profiles_runs_on_the_host(tmp_path):
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--summarize",
                        str(tmp_path)], capture_output=True, text=True, timeout=120)
    assert p.returncode == 0, p.stderr
