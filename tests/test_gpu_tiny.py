"""GPU parity on degenerate grids: single cells, one-cell-wide strips, grids
smaller than one marching tile or one vector unit, for every stencil kind.
Per-row kernels and local domains bit for bit against the oracle; converged
solves (global and Algorithm 1; FP64 and mixed, Jacobi and SGS; single and
batched) against the oracle's criterion and a dense
solve."""
import numpy as np
import pytest

import oracle
from paper_2001_01158_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2001_01158_amd import lcs  # noqa: E402

DEV = "cuda:0"
SHAPES = {
    W.KIND_5PT: [(1, 1, 1), (1, 6, 1), (6, 1, 1), (2, 2, 1), (3, 2, 1), (4, 5, 1), (8, 1, 1)],
    W.KIND_9PT: [(1, 1, 1), (1, 5, 1), (5, 1, 1), (2, 2, 1), (3, 4, 1), (4, 3, 1)],
    W.KIND_7PT: [(1, 1, 1), (1, 2, 3), (3, 1, 2), (2, 3, 1), (4, 2, 2), (1, 1, 5)],
    W.KIND_9N: [(1, 1, 1), (1, 4, 1), (4, 1, 1), (3, 3, 1), (4, 2, 1)],
}
CASES = [(k, s) for k, shapes in SHAPES.items() for s in shapes]


def say(*a):
    print("[case]", *a, flush=True)


def dev(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype).to(DEV)


def host(t):
    return t.detach().cpu().numpy()


def make(kind, dims, seed=0):
    nx, ny, nz = dims
    coef = lcs_coef(kind, dims, seed)
    Ah = oracle.csr_from_stencil(kind, nx, ny, nz, coef)
    rng = np.random.default_rng(seed)
    x_true = rng.random(Ah.n) + 0.5
    b = oracle.spmv(Ah, x_true)
    x0 = x_true * (1.0 + 0.2 * rng.random(Ah.n))
    A = lcs.matrix_from_numpy(kind, nx, ny, nz, coef, DEV)
    return Ah, A, b, x0


def name(kind, dims):
    return f"{W.KIND_NAMES[kind]}-{dims[0]}x{dims[1]}x{dims[2]}"


@pytest.mark.parametrize("kind,dims", CASES, ids=[name(k, s) for k, s in CASES])
def test_tiny_per_row_kernels_bitexact(kind, dims):
    Ah, A, b, x0 = make(kind, dims)
    say("tiny per-row", name(kind, dims))
    assert np.array_equal(host(lcs.residual(A, dev(b), dev(x0))), oracle.residual(Ah, b, x0))
    assert np.array_equal(host(lcs.gradient(A, dev(x0))), oracle.gradient(Ah, x0))
    y = torch.empty(A.n, dtype=torch.float64, device=DEV)
    lcs.spmv(A, dev(x0), y)
    assert np.array_equal(host(y), oracle.spmv(Ah, x0))
    x = dev(x0)
    lcs.gs_sweeps(A, dev(b), x, 2)
    assert np.array_equal(host(x), oracle.gs_sweeps(Ah, b, x0, 2))


@pytest.mark.parametrize("kind,dims", CASES, ids=[name(k, s) for k, s in CASES])
@pytest.mark.parametrize("mode,theta,e_max", [("residual", 0.3, 2), ("gradient", 0.3, 0)])
def test_tiny_local_domain_bitexact(kind, dims, mode, theta, e_max):
    Ah, A, b, x0 = make(kind, dims)
    say("tiny domain", name(kind, dims), mode)
    om = {"residual": oracle.MODE_RESIDUAL, "gradient": oracle.MODE_GRADIENT}[mode]
    idx, mask, st = lcs.build_local_domain(A, dev(b), dev(x0), mode, "relmax", theta, e_max,
                                           want_mask=True)
    d = oracle.build_local_domain(Ah, b, x0, om, theta, oracle.TH_RELMAX, e_max)
    assert st.K == d.K and np.array_equal(host(idx), d.idx)
    assert np.array_equal(host(mask), d.mask) and st.e_rounds == d.rounds


@pytest.mark.parametrize("kind,dims", CASES, ids=[name(k, s) for k, s in CASES])
def test_tiny_solves_converge(kind, dims):
    Ah, A, b, x0 = make(kind, dims)
    say("tiny solves", name(kind, dims))
    nb = np.linalg.norm(b)
    xd = np.linalg.solve(Ah.dense(), b)
    cond = np.linalg.cond(Ah.dense())
    variants = [dict()]
    if kind != W.KIND_9N:   # GMRES runs in FP64 with Jacobi or nothing
        variants += [dict(precond="rbsgs"), dict(precision="mixed"),
                     dict(precision="mixed", precond="rbsgs")]
    for extra in variants:
        o = lcs.Options(eps=1e-10, **extra)
        if extra.get("precision") == "mixed":
            A.coef32 = lcs.cast_coef(A)
        for call in ("global", "residual", "gradient"):
            x = dev(x0)
            if call == "global":
                lcs.solve_global(A, dev(b), x, o)
            else:
                lcs.solve_local_then_global(A, dev(b), x, call, "relmax", 0.3, 1, o)
            xg = host(x)
            what = (call, extra)
            assert np.linalg.norm(oracle.residual(Ah, b, xg)) <= 1.0001e-10 * nb, what
            assert np.linalg.norm(xg - xd) / np.linalg.norm(xd) <= max(10 * cond * 1e-10, 1e-12), what


@pytest.mark.parametrize("kind,dims", CASES, ids=[name(k, s) for k, s in CASES])
def test_tiny_batched(kind, dims):
    """Three systems of a degenerate grid in one batched launch (PCG for the
    symmetric kinds, GMRES for the non-symmetric one): each meets the
    criterion, with the oracle's domain size."""
    nx, ny, nz = dims
    say("tiny batched", name(kind, dims))
    cases = [make(kind, dims, seed=g) for g in range(3)]
    coef = np.stack([lcs_coef(kind, dims, g) for g in range(3)])
    b = np.stack([c[2] for c in cases])
    x0 = np.stack([c[3] for c in cases])
    A = lcs.BatchMatrix(kind, nx, ny, nz, dev(coef))
    x = dev(x0)
    sts = lcs.solve_local_then_global_batched(A, dev(b), x, "residual", "relmax", 0.3, 1,
                                              lcs.Options(eps=1e-10))
    xg = host(x)
    for g, (Ah, _, bg, x0g) in enumerate(cases):
        d = oracle.build_local_domain(Ah, bg, x0g, oracle.MODE_RESIDUAL, 0.3, oracle.TH_RELMAX, 1)
        assert sts[g].K == d.K
        assert np.linalg.norm(oracle.residual(Ah, bg, xg[g])) <= 1.0001e-10 * np.linalg.norm(bg)


def lcs_coef(kind, dims, seed):
    nx, ny, nz = dims
    if kind == W.KIND_9N:
        return W.assemble_9n(nx, ny, 0.25, speed=2.0 + 0.5 * seed)
    if kind == W.KIND_5PT:
        return W.assemble_5pt(W.lognormal_logk((ny, nx), 1.0, 40 + seed), 0.25)
    if kind == W.KIND_9PT:
        return W.assemble_9pt(nx, ny, 0.25, 100.0, 30.0)
    return W.assemble_7pt(W.lognormal_logk((nz, ny, nx), 1.0, 40 + seed), 0.25)
