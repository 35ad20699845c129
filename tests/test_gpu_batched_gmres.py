"""GPU parity of batched GMRES(m) on the non-symmetric nine-point kind (full
storage), one workgroup per system: every system against the oracle's
Algorithm 1 and global GMRES, GMRES trajectories at equal step caps across
restarts, the single-system calls of the library, and argument errors; on a
grid whose vectors fit in LDS and on one whose vectors do not."""
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
GRIDS = {"lds": (37, 29), "global": (97, 83)}   # 1073 and 8051 cells (LDS holds 7168)


def say(*a):
    print("[case]", *a, flush=True)


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64).to(DEV)


def host(t):
    return t.detach().cpu().numpy()


def gm_opts(**kw):
    return oracle.Options(krylov=oracle.KRYLOV_GMRES, **kw)


def case(g, dims):
    """System g: diffusion anisotropy and convection speed vary by group;
    x0 differs from the solution on a box."""
    nx, ny = dims
    coef = W.assemble_9n(nx, ny, 0.25, ratio=2.0 + g, speed=1.0 + 0.5 * g)
    Ah = oracle.csr_from_stencil(W.KIND_9N, nx, ny, 1, coef)
    rng = np.random.default_rng(500 + g)
    x_true = np.full(Ah.n, 0.1 + 0.01 * g)
    gr = x_true.reshape(ny, nx)
    gr[ny // 3: ny // 3 + 7, nx // 4: nx // 4 + 9] = 1.0
    b = oracle.spmv(Ah, x_true)
    x0 = x_true.copy()
    sl = (slice(ny // 5, ny // 5 + max(2, ny // 3)), slice(nx // 5, nx // 5 + max(2, nx // 3)))
    box = x0.reshape(ny, nx)[sl]
    x0.reshape(ny, nx)[sl] = box * (1.0 + 0.3 * rng.random(box.shape))
    return coef, Ah, b, x0


_DENSE = {}


def dense_solution(g, dims, Ah, b):
    """Dense solve of system g (cached: the parametrizations share systems)."""
    key = (g, dims)
    if key not in _DENSE:
        _DENSE[key] = np.linalg.solve(Ah.dense(), b)
    return _DENSE[key]


def make_batch(G, dims):
    cases = [case(g, dims) for g in range(G)]
    A = lcs.BatchMatrix(W.KIND_9N, dims[0], dims[1], 1, dev(np.stack([c[0] for c in cases])))
    return A, [c[1] for c in cases], np.stack([c[2] for c in cases]), np.stack([c[3] for c in cases])


@pytest.mark.parametrize("grid", list(GRIDS))
@pytest.mark.parametrize("mode,thresh,theta,e_max", [("residual", "relmax", 1e-3, 1),
                                                     ("residual", "paper", 1e-10, 1),
                                                     ("gradient", "relmax", 1e-4, 0)])
def test_batched_gmres_local_then_global_vs_oracle(grid, mode, thresh, theta, e_max):
    G = 3
    A, Ahs, b, x0 = make_batch(G, GRIDS[grid])
    say("batched gmres local_then_global", grid, mode, thresh)
    x = dev(x0)
    sts = lcs.solve_local_then_global_batched(A, dev(b), x, mode, thresh, theta, e_max,
                                              lcs.Options(eps=1e-10))
    xg = host(x)
    om = {"residual": oracle.MODE_RESIDUAL, "gradient": oracle.MODE_GRADIENT}[mode]
    ot = {"relmax": oracle.TH_RELMAX, "paper": oracle.TH_PAPER}[thresh]
    for g in range(G):
        xo, so, _ = oracle.local_then_global(Ahs[g], b[g], x0[g], om, theta, ot, e_max,
                                             gm_opts(eps=1e-10))
        if thresh == "paper":
            assert abs(sts[g].K - so.K) <= 2
        else:
            assert sts[g].K == so.K
        assert abs(sts[g].its_local - so.its_local) <= 2, (g, sts[g].its_local, so.its_local)
        nb = np.linalg.norm(b[g])
        assert np.linalg.norm(oracle.residual(Ahs[g], b[g], xg[g])) <= 1.0001e-10 * nb
        xd = dense_solution(g, GRIDS[grid], Ahs[g], b[g])
        err_g = np.linalg.norm(xg[g] - xd) / np.linalg.norm(xd)
        err_o = np.linalg.norm(xo - xd) / np.linalg.norm(xd)
        say(f"  g={g} K={sts[g].K} its={sts[g].its_local}+{sts[g].its_global} "
            f"(oracle {so.its_local}+{so.its_global}) err {err_g:.1e} / {err_o:.1e}")
        assert err_g <= max(10 * err_o, 1e-10)


@pytest.mark.parametrize("grid", list(GRIDS))
def test_batched_gmres_global_vs_oracle(grid):
    G = 3
    A, Ahs, b, x0 = make_batch(G, GRIDS[grid])
    say("batched gmres global", grid)
    x = dev(x0)
    sts = lcs.solve_global_batched(A, dev(b), x, lcs.Options(eps=1e-10))
    xg = host(x)
    for g in range(G):
        xo, so = oracle.solve_global(Ahs[g], b[g], x0[g], gm_opts(eps=1e-10))
        assert abs(sts[g].its_global - so.its_global) <= 2, (g, sts[g].its_global, so.its_global)
        nb = np.linalg.norm(b[g])
        assert np.linalg.norm(oracle.residual(Ahs[g], b[g], xg[g])) <= 1.0001e-10 * nb


@pytest.mark.parametrize("grid", list(GRIDS))
@pytest.mark.parametrize("pc", ["jacobi", "none"])
def test_batched_gmres_trajectory(grid, pc):
    """GMRES(4) stopped after k steps (k = 11 crosses two restarts) in the
    global solve, and Algorithm 1 with k steps in the local and in the global
    solve: rounding-level agreement with the oracle's modified Gram-Schmidt."""
    G = 2
    A, Ahs, b, x0 = make_batch(G, GRIDS[grid])
    opc = {"jacobi": oracle.PC_JACOBI, "none": oracle.PC_NONE}[pc]
    for k in (3, 11):
        say("batched gmres trajectory", grid, pc, k)
        o = lcs.Options(eps=1e-30, precond=pc, max_iter=k, restart=4, max_outer=0)
        x = dev(x0)
        with pytest.raises(lcs.LcsError) as e:
            lcs.solve_global_batched(A, dev(b), x, o)
        assert e.value.status == lcs.ENOCONV
        xg = host(x)
        for g in range(G):
            xk, _, itk, _ = oracle.gmres(Ahs[g], b[g], x0[g], opc, m=4, tol_abs=0.0, max_iter=k)
            assert itk == k
            rel = np.linalg.norm(xg[g] - xk) / np.linalg.norm(xk)
            assert rel <= 1e-10, (g, rel)
        x = dev(x0)
        with pytest.raises(lcs.LcsError) as e:
            lcs.solve_local_then_global_batched(A, dev(b), x, "residual", "relmax", 1e-3, 1, o)
        assert e.value.status == lcs.ENOCONV
        xg = host(x)
        for g in range(G):
            xo, so, _ = oracle.local_then_global(Ahs[g], b[g], x0[g], oracle.MODE_RESIDUAL, 1e-3,
                                                 oracle.TH_RELMAX, 1,
                                                 gm_opts(eps=1e-30, max_iter=k, gmres_m=4, pc=opc))
            rel = np.linalg.norm(xg[g] - xo) / np.linalg.norm(xo)
            assert rel <= 1e-10, (g, rel)


def test_batched_gmres_matches_single_system_calls():
    G = 4
    dims = GRIDS["lds"]
    A, Ahs, b, x0 = make_batch(G, dims)
    say("batched gmres vs single")
    xb = dev(x0)
    sts = lcs.solve_local_then_global_batched(A, dev(b), xb, "residual", "relmax", 1e-3, 2,
                                              lcs.Options(eps=1e-10))
    xbh = host(xb)
    for g in range(G):
        M = lcs.Matrix(W.KIND_9N, dims[0], dims[1], 1, A.coef[g].contiguous())
        xs = dev(x0[g])
        st = lcs.solve_local_then_global(M, dev(b[g]), xs, "residual", "relmax", 1e-3, 2,
                                         lcs.Options(eps=1e-10))
        assert st.K == sts[g].K and st.e_rounds == sts[g].e_rounds and st.tau == sts[g].tau
        assert abs(st.its_local - sts[g].its_local) <= 2
        nb = np.linalg.norm(b[g])
        assert np.linalg.norm(oracle.residual(Ahs[g], b[g], xbh[g])) <= 1.0001e-10 * nb


def test_batched_gmres_argument_errors():
    A, Ahs, b, x0 = make_batch(2, GRIDS["lds"])
    bb, x = dev(b), dev(x0)
    for opts in [lcs.Options(precision="mixed"), lcs.Options(precond="rbsgs"),
                 lcs.Options(restart=0), lcs.Options(restart=65)]:
        with pytest.raises(lcs.LcsError) as e:
            lcs.solve_global_batched(A, bb, x, opts)
        assert e.value.status == lcs.EINVAL
    assert np.array_equal(host(x), x0)


def test_multigroup_nonsym_batch_full_size():
    """The 64 non-symmetric group systems of 88 x 80 cells in one launch per
    method (global GMRES, gradient and residual domains): every system meets
    the criterion, recomputed by the oracle."""
    w = W.mg_batch_nonsym()
    say("multigroup nonsym 64 x 7040")
    A = lcs.BatchMatrix(W.KIND_9N, w.nx, w.ny, 1, dev(w.coef))
    Ahs = [oracle.csr_from_stencil(W.KIND_9N, w.nx, w.ny, 1, w.coef[g]) for g in range(w.G)]
    o = lcs.Options(eps=W.MG_EPS)
    calls = {
        "global": lambda x: lcs.solve_global_batched(A, dev(w.b), x, o),
        "gradient": lambda x: lcs.solve_local_then_global_batched(
            A, dev(w.b), x, "gradient", "relmax", W.MG_ALPHA, 0, o),
        "residual": lambda x: lcs.solve_local_then_global_batched(
            A, dev(w.b), x, "residual", "paper", W.MG_EPS, W.MG_E_MAX, o),
    }
    for name, call in calls.items():
        x = dev(w.x0)
        sts = call(x)
        xg = host(x)
        worst = 0.0
        for g in range(w.G):
            nb = np.linalg.norm(w.b[g])
            rel = np.linalg.norm(oracle.residual(Ahs[g], w.b[g], xg[g])) / nb
            worst = max(worst, rel)
            assert rel <= 1.0001 * W.MG_EPS, (name, g, rel)
        say(f"  {name}: worst relres {worst:.2e}, its of group 63: "
            f"{sts[-1].its_local}+{sts[-1].its_global}")


@pytest.mark.parametrize("call", ["global", "local_then_global"])
def test_batched_gmres_nonfinite_system_reported_others_solved(call):
    A, Ahs, b, x0 = make_batch(3, GRIDS["lds"])
    b = b.copy()
    b[1, 5] = np.nan
    say("batched gmres nonfinite", call)
    x = dev(x0)
    with pytest.raises(lcs.LcsError) as e:
        if call == "global":
            lcs.solve_global_batched(A, dev(b), x, lcs.Options(eps=1e-10))
        else:
            lcs.solve_local_then_global_batched(A, dev(b), x, "residual", "relmax", 1e-3, 1,
                                                lcs.Options(eps=1e-10))
    assert e.value.status == lcs.ENONFINITE
    assert "system 1" in str(e.value)
    xg = host(x)
    for g in (0, 2):
        nb = np.linalg.norm(b[g])
        assert np.linalg.norm(oracle.residual(Ahs[g], b[g], xg[g])) <= 1.0001e-10 * nb
