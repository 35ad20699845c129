"""Runtime behaviour of the library on the GPU: work follows the caller's
stream, one context serves systems of different kinds and sizes, CSR input
included (its workspace grows and is reused), with results bit-identical to
fresh contexts,
and repeated GMRES and batched solves are bitwise deterministic."""
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


def say(*a):
    print("[case]", *a, flush=True)


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64).to(DEV)


def host(t):
    return t.detach().cpu().numpy()


def case(kind, dims, seed=0):
    """Operator, b and x0 (x_true perturbed on a box) of one system."""
    nx, ny, nz = dims
    if kind == W.KIND_5PT:
        coef = W.assemble_5pt(W.lognormal_logk((ny, nx), 1.0, 60 + seed), 0.25)
    elif kind == W.KIND_9PT:
        coef = W.assemble_9pt(nx, ny, 0.25, 100.0, 30.0)
    elif kind == W.KIND_7PT:
        coef = W.assemble_7pt(W.lognormal_logk((nz, ny, nx), 1.0, 60 + seed), 0.25)
    else:
        coef = W.assemble_9n(nx, ny, 0.25, speed=2.0)
    Ah = oracle.csr_from_stencil(kind, nx, ny, nz, coef)
    rng = np.random.default_rng(seed)
    x_true = np.full(Ah.n, 0.1)
    g = x_true.reshape(nz, ny, nx)
    g[:, ny // 3: ny // 3 + max(1, ny // 4), nx // 4: nx // 4 + max(1, nx // 4)] = 1.0
    b = oracle.spmv(Ah, x_true)
    x0 = x_true * (1.0 + 0.2 * rng.random(Ah.n))
    return coef, Ah, b, x0


def solve(kind, dims, coef, b, x0, ctx, opts=None):
    A = lcs.matrix_from_numpy(kind, *dims, coef, DEV)
    x = dev(x0)
    st = lcs.solve_local_then_global(A, dev(b), x, "residual", "relmax", 1e-3, 1,
                                     opts or lcs.Options(eps=1e-10), ctx=ctx)
    return host(x), st


def test_side_stream_matches_default_stream():
    """A solve issued under a non-default torch stream runs on that stream
    and gives the default stream's result bit for bit."""
    dims = (93, 71, 1)
    coef, Ah, b, x0 = case(W.KIND_5PT, dims)
    say("side stream")
    ctx = lcs.Context()
    x_def, st_def = solve(W.KIND_5PT, dims, coef, b, x0, ctx)
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        A = lcs.matrix_from_numpy(W.KIND_5PT, *dims, coef, DEV)
        bb, x = dev(b), dev(x0)
        st = lcs.solve_local_then_global(A, bb, x, "residual", "relmax", 1e-3, 1,
                                         lcs.Options(eps=1e-10), ctx=ctx)
    side.synchronize()
    assert np.array_equal(host(x), x_def)
    assert (st.K, st.its_local, st.its_global) == (st_def.K, st_def.its_local, st_def.its_global)
    assert np.linalg.norm(oracle.residual(Ah, b, host(x))) <= 1.0001e-10 * np.linalg.norm(b)


def test_context_reuse_across_kinds_and_sizes():
    """One context through systems of growing and shrinking sizes and all
    four kinds (the workspace grows and is reused), then the first system
    again: every result equals a fresh context's bit for bit."""
    seq = [(W.KIND_9PT, (83, 67, 1)), (W.KIND_5PT, (20, 13, 1)), (W.KIND_7PT, (23, 19, 17)),
           (W.KIND_9N, (37, 29, 1)), (W.KIND_5PT, (256, 200, 1)), (W.KIND_9PT, (83, 67, 1))]
    shared = lcs.Context()
    for k, (kind, dims) in enumerate(seq):
        say("context reuse", k, W.KIND_NAMES[kind], dims)
        coef, Ah, b, x0 = case(kind, dims, seed=k)
        xs, sts = solve(kind, dims, coef, b, x0, shared)
        xf, stf = solve(kind, dims, coef, b, x0, lcs.Context())
        assert np.array_equal(xs, xf)
        assert (sts.K, sts.its_local, sts.its_global) == (stf.K, stf.its_local, stf.its_global)
        assert np.linalg.norm(oracle.residual(Ah, b, xs)) <= 1.0001e-10 * np.linalg.norm(b)


def test_gmres_run_twice_bitwise():
    dims = (64, 48, 1)
    coef, Ah, b, x0 = case(W.KIND_9N, dims)
    say("gmres run twice")
    out = [solve(W.KIND_9N, dims, coef, b, x0, lcs.Context(), lcs.Options(eps=1e-10, restart=12))[0]
           for _ in range(2)]
    assert np.array_equal(out[0], out[1])


def test_batched_run_twice_bitwise():
    dims = (41, 23, 1)
    say("batched run twice")
    cases = [case(W.KIND_5PT, dims, seed=g) for g in range(5)]
    A = lcs.BatchMatrix(W.KIND_5PT, *dims, dev(np.stack([c[0] for c in cases])))
    b = dev(np.stack([c[2] for c in cases]))
    x0 = np.stack([c[3] for c in cases])
    out = []
    for _ in range(2):
        x = dev(x0)
        lcs.solve_local_then_global_batched(A, b, x, "residual", "relmax", 1e-3, 1,
                                            lcs.Options(eps=1e-10))
        out.append(host(x))
    assert np.array_equal(out[0], out[1])


def test_context_reuse_with_csr_input():
    """One context through CSR matrices of ELL widths 16 and 5 and a stencil
    in between, then the first CSR matrix again: each result equals a fresh
    context's bit for bit (the ELL copy is rebuilt for every call)."""
    def csr_case(nx, ny, seed, **kw):
        rp, col, val = W.irregular_spd(nx, ny, seed, **kw)
        colour, nc = W.greedy_colouring(rp, col)
        Ah = oracle.CSR(nx * ny, rp, col, val, colour, nc)
        A = lcs.CsrMatrix(dev(rp).to(torch.int32), dev(col).to(torch.int32), dev(val),
                          dev(colour).to(torch.uint8), nc)
        rng = np.random.default_rng(seed)
        x_true = np.full(Ah.n, 0.1)
        x_true[: Ah.n // 5] = 1.0
        b = oracle.spmv(Ah, x_true)
        return Ah, A, b, x_true * (1.0 + 0.2 * rng.random(Ah.n))

    def run(A, b, x0, ctx):
        x = dev(x0)
        st = lcs.solve_local_then_global(A, dev(b), x, "residual", "relmax", 1e-3, 1,
                                         lcs.Options(eps=1e-10, precond="rbsgs"), ctx=ctx)
        return host(x), (st.K, st.its_local, st.its_global)

    first = csr_case(47, 39, 1)
    seq = [first, csr_case(31, 23, 2, p_diag=0.0, p_long=0.0), "stencil", first]
    shared = lcs.Context()
    for k, item in enumerate(seq):
        say("context reuse with csr", k)
        if item == "stencil":
            coef, Ah, b, x0 = case(W.KIND_5PT, (64, 40, 1), seed=k)
            xs, _ = solve(W.KIND_5PT, (64, 40, 1), coef, b, x0, shared)
            xf, _ = solve(W.KIND_5PT, (64, 40, 1), coef, b, x0, lcs.Context())
            assert np.array_equal(xs, xf)
            continue
        Ah, A, b, x0 = item
        xs, ss = run(A, b, x0, shared)
        xf, sf = run(A, b, x0, lcs.Context())
        assert np.array_equal(xs, xf) and ss == sf
        assert np.linalg.norm(oracle.residual(Ah, b, xs)) <= 1.0001e-10 * np.linalg.norm(b)
