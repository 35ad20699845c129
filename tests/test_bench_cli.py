"""bench.py's parts that need no GPU: more than one GPU is refused with a
message (the implementation runs on one GPU), the rocprofv3 summarizer runs on
the host, and the CSR built for the library SpMV yardstick is the oracle's CSR
of the same nine-point stencil."""
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


def test_csr_yardstick_matrix_is_the_oracles_csr():
    import numpy as np
    import pytest
    torch = pytest.importorskip("torch")
    sys.path.insert(0, ROOT)
    import bench
    import oracle
    from paper_2001_01158_amd import workloads as W
    for nx, ny in [(7, 5), (8, 6), (1, 4), (5, 1)]:
        c = W.assemble_9pt(nx, ny, 0.25, 100.0, 30.0)
        crow, col, val = bench.csr_from_nine_point(torch.as_tensor(c).reshape(5, -1), nx, ny)
        A = oracle.csr_from_stencil(W.KIND_9PT, nx, ny, 1, c)
        assert np.array_equal(crow.numpy(), A.rp)
        assert np.array_equal(col.numpy(), A.col)
        assert np.array_equal(val.numpy(), A.val)
