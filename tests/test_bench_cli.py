"""bench.py's parts that need no GPU: more than one GPU is refused with a
message (the implementation runs on one GPU), the rocprofv3 summarizer runs on
the host, the CSR built for the library SpMV yardstick is the oracle's CSR
of the same nine-point stencil, and the CSR input of bench.py --csr is the
oracle's CSR of each stencil kind."""
import json
import os
import subprocess
import sys

import numpy as np
import pytest

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


@pytest.mark.parametrize("kind,dims", [(0, (13, 9, 1)), (1, (11, 8, 1)), (2, (7, 6, 5)), (3, (10, 7, 1))])
def test_bench_csr_input_is_the_oracles_csr(kind, dims):
    """The CSR that bench.py --csr hands to the library equals the oracle's
    CSR of the same stencil (pattern, order and values) and the oracle's
    grid colouring."""
    import bench
    import oracle
    from paper_2001_01158_amd import workloads as W
    nx, ny, nz = dims
    if kind == W.KIND_5PT:
        coef = W.assemble_5pt(W.lognormal_logk((ny, nx), 1.0, 3), 0.25)
    elif kind == W.KIND_9PT:
        coef = W.assemble_9pt(nx, ny, 0.25, 100.0, 30.0)
    elif kind == W.KIND_7PT:
        coef = W.assemble_7pt(W.lognormal_logk((nz, ny, nx), 1.0, 3), 0.25)
    else:
        coef = W.assemble_9n(nx, ny, 0.25, speed=2.0)
    rp, col, val, colour, nc = bench.csr_arrays(kind, nx, ny, nz, coef)
    Ah = oracle.csr_from_stencil(kind, nx, ny, nz, coef)
    assert np.array_equal(rp, Ah.rp) and np.array_equal(col, Ah.col)
    assert np.array_equal(val, Ah.val)
    assert np.array_equal(colour, Ah.colour) and nc == Ah.ncolours
