"""GPU parity for the non-symmetric nine-point operator (full storage) and
its GMRES(m) solves: per-row kernels and the local domain bit for bit, the
GMRES trajectory at equal step counts (across restarts), converged solves of
Algorithm 1 against the oracle, argument errors, and a 1024^2 system."""
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
GRIDS = {"odd": (37, 29), "even": (40, 23)}


def say(*a):
    print("[case]", *a, flush=True)


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64).to(DEV)


def host(t):
    return t.detach().cpu().numpy()


def make_case(grid, seed=0, dt=4.0, speed=2.0):
    nx, ny = GRIDS[grid] if isinstance(grid, str) else grid
    coef = W.assemble_9n(nx, ny, 1.0 / dt, speed=speed)
    Ah = oracle.csr_from_stencil(W.KIND_9N, nx, ny, 1, coef)
    n = nx * ny
    rng = np.random.default_rng(seed)
    x_true = np.full(n, 0.1)
    g = x_true.reshape(ny, nx)
    g[ny // 3: ny // 3 + 7, nx // 4: nx // 4 + 9] = 1.0
    b = oracle.spmv(Ah, x_true)
    x0 = x_true.copy()
    sl = (slice(ny // 5, ny // 5 + max(2, ny // 2)), slice(nx // 5, nx // 5 + max(2, nx // 2)))
    box = x0.reshape(ny, nx)[sl]
    x0.reshape(ny, nx)[sl] = box * (1.0 + 0.3 * rng.random(box.shape))
    A = lcs.matrix_from_numpy(lcs.STENCIL9N_2D, nx, ny, 1, coef, DEV)
    return coef, Ah, A, b, x0


def gm_opts(**kw):
    return oracle.Options(krylov=oracle.KRYLOV_GMRES, **kw)


@pytest.mark.parametrize("grid", list(GRIDS))
def test_nonsym_per_row_bitexact(grid):
    coef, Ah, A, b, x0 = make_case(grid)
    say("nonsym per-row", grid)
    assert np.array_equal(host(lcs.residual(A, dev(b), dev(x0))), oracle.residual(Ah, b, x0))
    assert np.array_equal(host(lcs.gradient(A, dev(x0))), oracle.gradient(Ah, x0))
    y = torch.empty(A.n, dtype=torch.float64, device=DEV)
    lcs.spmv(A, dev(x0), y)
    assert np.array_equal(host(y), oracle.spmv(Ah, x0))
    x = dev(x0)
    lcs.gs_sweeps(A, dev(b), x, 2)
    assert np.array_equal(host(x), oracle.gs_sweeps(Ah, b, x0, 2))


@pytest.mark.parametrize("grid", list(GRIDS))
@pytest.mark.parametrize("mode,theta,e_max", [("residual", 1e-3, 1), ("residual", 1e-3, 3),
                                              ("gradient", 1e-4, 0)])
def test_nonsym_local_domain_and_gather_bitexact(grid, mode, theta, e_max):
    coef, Ah, A, b, x0 = make_case(grid)
    say("nonsym domain", grid, mode, e_max)
    om = {"residual": oracle.MODE_RESIDUAL, "gradient": oracle.MODE_GRADIENT}[mode]
    idx, mask, st = lcs.build_local_domain(A, dev(b), dev(x0), mode, "relmax", theta, e_max,
                                           want_mask=True)
    d = oracle.build_local_domain(Ah, b, x0, om, theta, oracle.TH_RELMAX, e_max)
    assert st.K == d.K and np.array_equal(host(idx), d.idx)
    assert np.array_equal(host(mask), d.mask) and st.e_rounds == d.rounds
    rp, col, val = lcs.gather_restricted(A, idx)
    B = oracle.restricted(Ah, d.idx)
    assert np.array_equal(host(rp).astype(np.int64), B.rp)
    assert np.array_equal(host(col), B.col) and np.array_equal(host(val), B.val)


@pytest.mark.parametrize("grid", list(GRIDS))
@pytest.mark.parametrize("pc", ["jacobi", "none"])
def test_nonsym_gmres_global_parity(grid, pc):
    coef, Ah, A, b, x0 = make_case(grid)
    say("nonsym global gmres", grid, pc)
    opc = {"jacobi": oracle.PC_JACOBI, "none": oracle.PC_NONE}[pc]
    xo, so = oracle.solve_global(Ah, b, x0, gm_opts(eps=1e-10, pc=opc))
    assert so.status == oracle.OK
    x = dev(x0)
    st = lcs.solve_global(A, dev(b), x, lcs.Options(eps=1e-10, precond=pc))
    nb = np.linalg.norm(b)
    assert np.linalg.norm(oracle.residual(Ah, b, host(x))) <= 1.0001e-10 * nb
    assert abs(st.its_global - so.its_global) <= 2
    # trajectory: both stop after exactly k Arnoldi steps (restart 10, so 25
    # steps cross two restarts); CGS2 against the oracle's modified
    # Gram-Schmidt differs only in rounding
    for k in (3, 9, 25):
        xk, stk, itk, _ = oracle.gmres(Ah, b, x0, opc, m=10, tol_abs=0.0, max_iter=k)
        assert itk == k
        xg = dev(x0)
        with pytest.raises(lcs.LcsError) as e:
            lcs.solve_global(A, dev(b), xg, lcs.Options(eps=1e-30, precond=pc, max_iter=k,
                                                         restart=10, max_outer=0))
        assert e.value.status == lcs.ENOCONV
        rel = np.linalg.norm(host(xg) - xk) / np.linalg.norm(xk)
        say(f"  k={k} rel={rel:.2e}")
        assert rel <= 1e-10


@pytest.mark.parametrize("grid", list(GRIDS))
@pytest.mark.parametrize("mode,thresh,theta", [("residual", "relmax", 1e-3),
                                               ("residual", "paper", 1e-10),
                                               ("gradient", "relmax", 1e-4)])
def test_nonsym_local_then_global_parity(grid, mode, thresh, theta):
    coef, Ah, A, b, x0 = make_case(grid)
    say("nonsym local_then_global", grid, mode, thresh)
    om = {"residual": oracle.MODE_RESIDUAL, "gradient": oracle.MODE_GRADIENT}[mode]
    ot = {"relmax": oracle.TH_RELMAX, "paper": oracle.TH_PAPER}[thresh]
    xo, so, dom = oracle.local_then_global(Ah, b, x0, om, theta, ot, 1, gm_opts(eps=1e-10))
    x = dev(x0)
    st = lcs.solve_local_then_global(A, dev(b), x, mode, thresh, theta, 1, lcs.Options(eps=1e-10))
    if thresh == "paper":
        assert abs(st.K - so.K) <= 2
    else:
        assert st.K == so.K
    assert abs(st.its_local - so.its_local) <= 2
    nb = np.linalg.norm(b)
    xg = host(x)
    assert np.linalg.norm(oracle.residual(Ah, b, xg)) <= 1.0001e-10 * nb
    xd = np.linalg.solve(Ah.dense(), b)
    err_g = np.linalg.norm(xg - xd) / np.linalg.norm(xd)
    err_o = np.linalg.norm(xo - xd) / np.linalg.norm(xd)
    say(f"  K={st.K} its={st.its_local}+{st.its_global} err {err_g:.1e} / {err_o:.1e}")
    assert err_g <= max(10 * err_o, 1e-10)


def test_nonsym_argument_errors():
    coef, Ah, A, b, x0 = make_case("odd")
    bb, x = dev(b), dev(x0)
    for opts in [lcs.Options(precision="mixed"), lcs.Options(precond="rbsgs"),
                 lcs.Options(restart=0), lcs.Options(restart=65)]:
        with pytest.raises(lcs.LcsError) as e:
            lcs.solve_global(A, bb, x, opts)
        assert e.value.status == lcs.EINVAL
    Ab = lcs.BatchMatrix(lcs.STENCIL9N_2D, A.nx, A.ny, 1, A.coef.reshape(1, 9, A.n).contiguous())
    with pytest.raises(lcs.LcsError) as e:   # batched GMRES runs in FP64
        lcs.solve_global_batched(Ab, bb.reshape(1, -1).contiguous(), x.reshape(1, -1),
                                 lcs.Options(precision="mixed"))
    assert e.value.status == lcs.EINVAL
    assert np.array_equal(host(x), x0)


def test_nonsym_full_size_1024():
    """1024^2 non-symmetric system: the local domain bit for bit against the
    oracle, and the solution of Algorithm 1 (GMRES) meeting the criterion as
    recomputed by the oracle."""
    n1 = 1024
    coef, Ah, A, b, x0 = make_case((n1, n1), seed=4)
    say("nonsym 1024^2")
    idx, _, st = lcs.build_local_domain(A, dev(b), dev(x0), "residual", "relmax", 1e-3, 1)
    d = oracle.build_local_domain(Ah, b, x0, oracle.MODE_RESIDUAL, 1e-3, oracle.TH_RELMAX, 1)
    assert st.K == d.K and np.array_equal(host(idx), d.idx)
    x = dev(x0)
    st = lcs.solve_local_then_global(A, dev(b), x, "residual", "paper", 1e-10, 1,
                                     lcs.Options(eps=1e-10))
    nb = np.linalg.norm(b)
    assert np.linalg.norm(oracle.residual(Ah, b, host(x))) <= 1.0001e-10 * nb
    say(f"  K={st.K} its={st.its_local}+{st.its_global}")


@pytest.mark.parametrize("grid", list(GRIDS))
def test_nonsym_solve_local_trajectory_parity(grid):
    """Steps 3-7 of Algorithm 1 on a caller-supplied domain: GMRES on B
    stopped after the same number of steps on both sides (restart 4, so the
    cap of 11 crosses two restarts), then assembly and one Gauss-Seidel
    sweep: rounding-level agreement with the oracle."""
    coef, Ah, A, b, x0 = make_case(grid)
    say("nonsym solve_local", grid)
    d = oracle.build_local_domain(Ah, b, x0, oracle.MODE_RESIDUAL, 1e-4, oracle.TH_RELMAX, 1)
    assert 0 < d.K < A.n
    oo = gm_opts(eps=1e-10, max_iter=11, n_smooth=1, gmres_m=4)
    xo, so = oracle.solve_local(Ah, b, x0, d.idx, oo)
    x = dev(x0)
    st = lcs.solve_local(A, dev(b), x, torch.as_tensor(d.idx, dtype=torch.int32).to(DEV),
                         lcs.Options(eps=1e-10, max_iter=11, n_smooth=1, restart=4))
    assert st.its_local == so.its_local == 11
    rel = np.linalg.norm(host(x) - xo) / np.linalg.norm(xo)
    assert rel <= 1e-12, rel


@pytest.mark.parametrize("grid", list(GRIDS))
def test_nonsym_spmv_fp32(grid):
    """FP32 SpMV of the full-storage operator: within the FP32 rounding bound
    of a 9-term fused sum of the FP64 product of the same FP32-rounded
    inputs."""
    coef, Ah, A, b, x0 = make_case(grid)
    A.coef32 = lcs.cast_coef(A)
    c32 = host(A.coef32).astype(np.float64)
    np.testing.assert_array_equal(c32, coef.astype(np.float32).astype(np.float64))
    x32 = torch.as_tensor(x0, dtype=torch.float32).to(DEV)
    y = torch.empty(A.n, dtype=torch.float32, device=DEV)
    lcs.spmv(A, x32, y)
    A32h = oracle.csr_from_stencil(W.KIND_9N, A.nx, A.ny, 1, c32)
    xr = host(x32).astype(np.float64)
    ref = oracle.spmv(A32h, xr)
    absA = oracle.CSR(A32h.n, A32h.rp, A32h.col, np.abs(A32h.val))
    bound = 9 * 2.0 ** -24 * oracle.spmv(absA, np.abs(xr)) + 1e-30
    assert np.all(np.abs(host(y).astype(np.float64) - ref) <= bound)
