"""GPU parity of the batched solves (G systems on one grid, one workgroup
each): every system against the oracle's Algorithm 1 / global PCG, against
the single-system calls of the library, trajectories at equal iteration caps,
and the edge cases of a batch (a converged system, an all-zero system, a
non-finite system among good ones, grids smaller than a workgroup)."""
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
KIND = {"5pt": W.KIND_5PT, "9pt": W.KIND_9PT, "7pt": W.KIND_7PT}
DIMS = {"5pt": (41, 23, 1), "9pt": (37, 29, 1), "7pt": (13, 11, 9)}
MODES = {"residual": oracle.MODE_RESIDUAL, "gradient": oracle.MODE_GRADIENT}
THRESH = {"relmax": oracle.TH_RELMAX, "paper": oracle.TH_PAPER, "abs": oracle.TH_ABS}


def say(*a):
    print("[case]", *a, flush=True)


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64).to(DEV)


def host(t):
    return t.detach().cpu().numpy()


def group_case(name, g, dims=None, dt=4.0):
    """One system of a batch: operator, b, x0 (the previous state differs from
    the solution on a box), seeded per group."""
    kind = KIND[name]
    nx, ny, nz = dims or DIMS[name]
    seed = 300 + 17 * g
    if kind == W.KIND_5PT:
        coef = W.assemble_5pt(W.lognormal_logk((ny, nx), 1.0, seed), 1.0 / dt)
    elif kind == W.KIND_7PT:
        coef = W.assemble_7pt(W.lognormal_logk((nz, ny, nx), 1.0, seed), 1.0 / dt)
    else:
        coef = W.assemble_9pt(nx, ny, 1.0 / dt, 100.0, 30.0) * (1.0 + 0.5 * g)
    n = nx * ny * nz
    rng = np.random.default_rng(seed)
    x_true = np.full(n, 0.1) + 0.01 * g
    gr = x_true.reshape(nz, ny, nx)
    gr[nz // 3: nz // 3 + max(1, nz // 3), ny // 3: ny // 3 + 7, nx // 4: nx // 4 + 9] = 1.0
    Ah = oracle.csr_from_stencil(kind, nx, ny, nz, coef)
    b = oracle.spmv(Ah, x_true)
    x0 = x_true.copy()
    sl = (slice(0, nz), slice(ny // 4, ny // 4 + max(2, ny // 3)), slice(nx // 5, nx // 5 + max(2, nx // 3)))
    box = x0.reshape(nz, ny, nx)[sl]
    x0.reshape(nz, ny, nx)[sl] = box * (1.0 + 0.3 * rng.random(box.shape))
    return coef, Ah, b, x0


def make_batch(name, G, dims=None):
    cases = [group_case(name, g, dims) for g in range(G)]
    nx, ny, nz = dims or DIMS[name]
    coef = np.stack([c[0] for c in cases])
    A = lcs.BatchMatrix(KIND[name], nx, ny, nz, dev(coef))
    b = np.stack([c[2] for c in cases])
    x0 = np.stack([c[3] for c in cases])
    return A, [c[1] for c in cases], b, x0


@pytest.mark.parametrize("name", ["5pt", "9pt", "7pt"])
@pytest.mark.parametrize("mode,thresh,theta,e_max", [("residual", "relmax", 1e-3, 1),
                                                     ("residual", "relmax", 1e-3, 3),
                                                     ("residual", "paper", 1e-10, 1),
                                                     ("gradient", "relmax", 1e-4, 0)])
def test_batched_local_then_global_vs_oracle(name, mode, thresh, theta, e_max):
    G = 4
    say("batched local_then_global", name, mode, thresh, theta, e_max)
    A, Ahs, b, x0 = make_batch(name, G)
    x = dev(x0)
    sts = lcs.solve_local_then_global_batched(A, dev(b), x, mode, thresh, theta, e_max,
                                              lcs.Options(eps=1e-10))
    xg = host(x)
    for g in range(G):
        xo, so, dom = oracle.local_then_global(Ahs[g], b[g], x0[g], MODES[mode], theta,
                                               THRESH[thresh], e_max, oracle.Options(eps=1e-10))
        st = sts[g]
        if thresh == "paper":
            assert abs(st.K - so.K) <= 2, (g, st.K, so.K)
        else:
            assert st.K == so.K, (g, st.K, so.K)
            assert st.e_rounds == dom.rounds
        assert abs(st.its_local - so.its_local) <= 1
        nb = np.linalg.norm(b[g])
        assert np.linalg.norm(oracle.residual(Ahs[g], b[g], xg[g])) <= 1.0001e-10 * nb
        xd = oracle.pcg(Ahs[g], b[g], xo, oracle.PC_JACOBI, 1e-14 * nb, 5000)[0]
        err_g = np.linalg.norm(xg[g] - xd) / np.linalg.norm(xd)
        err_o = np.linalg.norm(xo - xd) / np.linalg.norm(xd)
        say(f"  g={g} K={st.K} its={st.its_local}+{st.its_global} err {err_g:.1e} / {err_o:.1e}")
        assert err_g <= max(10 * err_o, 1e-10)


@pytest.mark.parametrize("name,pc", [("5pt", "jacobi"), ("9pt", "jacobi"), ("7pt", "jacobi"),
                                     ("5pt", "none")])
def test_batched_global_vs_oracle(name, pc):
    G = 3
    say("batched global", name, pc)
    A, Ahs, b, x0 = make_batch(name, G)
    x = dev(x0)
    sts = lcs.solve_global_batched(A, dev(b), x, lcs.Options(eps=1e-10, precond=pc))
    xg = host(x)
    opc = {"jacobi": oracle.PC_JACOBI, "none": oracle.PC_NONE}[pc]
    for g in range(G):
        xo, so = oracle.solve_global(Ahs[g], b[g], x0[g], oracle.Options(eps=1e-10, pc=opc))
        assert abs(sts[g].its_global - so.its_global) <= 1
        assert sts[g].K == 0 and sts[g].its_local == 0
        nb = np.linalg.norm(b[g])
        assert np.linalg.norm(oracle.residual(Ahs[g], b[g], xg[g])) <= 1.0001e-10 * nb


@pytest.mark.parametrize("name", ["5pt", "9pt", "7pt"])
def test_batched_trajectory_parity(name):
    """Whole Algorithm 1 with an iteration cap m on both the local and the
    global PCG (both sides stop at m): the batched result agrees with the
    oracle's to rounding, which a wrong index, sign or coefficient anywhere in
    the flow would break at O(1)."""
    G = 3
    A, Ahs, b, x0 = make_batch(name, G)
    for m in (3, 9):
        say("batched trajectory", name, m)
        x = dev(x0)
        with pytest.raises(lcs.LcsError) as e:
            lcs.solve_local_then_global_batched(A, dev(b), x, "residual", "relmax", 1e-3, 1,
                                                lcs.Options(eps=1e-30, max_iter=m, max_outer=0))
        assert e.value.status == lcs.ENOCONV
        xg = host(x)
        for g in range(G):
            xo, so, _ = oracle.local_then_global(Ahs[g], b[g], x0[g], oracle.MODE_RESIDUAL, 1e-3,
                                                 oracle.TH_RELMAX, 1,
                                                 oracle.Options(eps=1e-30, max_iter=m))
            rel = np.linalg.norm(xg[g] - xo) / np.linalg.norm(xo)
            assert rel <= 1e-10, (g, rel)


@pytest.mark.parametrize("name", ["5pt", "9pt", "7pt"])
def test_batched_matches_single_system_calls(name):
    G = 4
    say("batched vs single", name)
    A, Ahs, b, x0 = make_batch(name, G)
    xb = dev(x0)
    sts = lcs.solve_local_then_global_batched(A, dev(b), xb, "residual", "relmax", 1e-3, 2,
                                              lcs.Options(eps=1e-10))
    for g in range(G):
        M = lcs.Matrix(A.kind, A.nx, A.ny, A.nz, A.coef[g].contiguous())
        xs = dev(x0[g])
        st = lcs.solve_local_then_global(M, dev(b[g]), xs, "residual", "relmax", 1e-3, 2,
                                         lcs.Options(eps=1e-10))
        assert st.K == sts[g].K and st.e_rounds == sts[g].e_rounds and st.tau == sts[g].tau
        assert abs(st.its_local - sts[g].its_local) <= 1


def test_batched_edge_systems():
    """A batch of: a converged system (returned unchanged, K = 0), an all-zero
    system (b = 0, x0 = 0), and an ordinary one, on a grid smaller than a
    workgroup (3 x 2 cells) and on a ragged one."""
    for dims in [(3, 2, 1), (45, 31, 1)]:
        say("batched edge systems", dims)
        cases = [group_case("5pt", g, dims) for g in range(3)]
        coef = np.stack([c[0] for c in cases])
        b = np.stack([c[2] for c in cases])
        x0 = np.stack([c[3] for c in cases])
        Ah0 = cases[0][1]
        nb0 = np.linalg.norm(b[0])
        x0[0] = oracle.pcg(Ah0, b[0], x0[0], oracle.PC_JACOBI, 1e-14 * nb0, 5000)[0]
        b[1] = 0.0
        x0[1] = 0.0
        A = lcs.BatchMatrix(W.KIND_5PT, *dims, dev(coef))
        x = dev(x0)
        sts = lcs.solve_local_then_global_batched(A, dev(b), x, "residual", "paper", 1e-10, 1,
                                                  lcs.Options(eps=1e-10))
        xg = host(x)
        assert sts[0].K == 0 and sts[0].its_local == 0 and sts[0].its_global == 0
        assert np.array_equal(xg[0], x0[0])
        assert sts[1].K == 0 and np.array_equal(xg[1], np.zeros_like(xg[1]))
        nb2 = np.linalg.norm(b[2])
        assert np.linalg.norm(oracle.residual(cases[2][1], b[2], xg[2])) <= 1.0001e-10 * nb2


def test_batched_nonfinite_system_reported_others_solved():
    A, Ahs, b, x0 = make_batch("5pt", 3)
    b = b.copy()
    b[1, 5] = np.nan
    x = dev(x0)
    with pytest.raises(lcs.LcsError) as e:
        lcs.solve_local_then_global_batched(A, dev(b), x, "residual", "relmax", 1e-3, 1,
                                            lcs.Options(eps=1e-10))
    assert e.value.status == lcs.ENONFINITE
    assert "system 1" in str(e.value)
    xg = host(x)
    for g in (0, 2):
        nb = np.linalg.norm(b[g])
        assert np.linalg.norm(oracle.residual(Ahs[g], b[g], xg[g])) <= 1.0001e-10 * nb


def test_batched_argument_errors():
    A, Ahs, b, x0 = make_batch("9pt", 2)
    bb, x = dev(b), dev(x0)
    for opts in [lcs.Options(precision="mixed"), lcs.Options(precond="rbsgs")]:
        with pytest.raises(lcs.LcsError) as e:
            lcs.solve_local_then_global_batched(A, bb, x, "residual", "relmax", 1e-3, 1, opts)
        assert e.value.status == lcs.EINVAL
    with pytest.raises(lcs.LcsError) as e:
        lcs.solve_local_then_global_batched(A, bb, x, "residual", "relmax", -1.0, 1)
    assert e.value.status == lcs.EINVAL
    with pytest.raises(ValueError):
        lcs.solve_global_batched(A, bb[:1], x)
    assert np.array_equal(host(x), x0)


def test_multigroup_batch_full_size():
    """The 64 group systems of the multi-group source iteration (88 x 80 =
    7040 cells, nine-point): every system meets the criterion (recomputed by
    the oracle); sampled groups match the oracle's Algorithm 1 (gradient
    domain, alpha = 1e-10, and residual domain, E_max = 1) and global PCG."""
    w = W.mg_batch()
    A = lcs.BatchMatrix(W.KIND_9PT, w.nx, w.ny, 1, dev(w.coef))
    o = lcs.Options(eps=W.MG_EPS)
    runs = {
        "gradient": lambda x: lcs.solve_local_then_global_batched(
            A, dev(w.b), x, "gradient", "relmax", W.MG_ALPHA, 0, o),
        "residual": lambda x: lcs.solve_local_then_global_batched(
            A, dev(w.b), x, "residual", "paper", W.MG_EPS, W.MG_E_MAX, o),
        "global": lambda x: lcs.solve_global_batched(A, dev(w.b), x, o),
    }
    for name, run in runs.items():
        say("multigroup batch", name)
        x = dev(w.x0)
        sts = run(x)
        xg = host(x)
        for g in range(w.G):
            Ah = oracle.csr_from_stencil(W.KIND_9PT, w.nx, w.ny, 1, w.coef[g])
            nb = np.linalg.norm(w.b[g])
            assert np.linalg.norm(oracle.residual(Ah, w.b[g], xg[g])) <= 1.0001 * W.MG_EPS * nb, g
            if g not in (0, 10, 41, 63):
                continue
            oo = oracle.Options(eps=W.MG_EPS)
            if name == "global":
                xo, so = oracle.solve_global(Ah, w.b[g], w.x0[g], oo)
                assert abs(sts[g].its_global - so.its_global) <= 1
                continue
            if name == "gradient":
                xo, so, dom = oracle.local_then_global(Ah, w.b[g], w.x0[g], oracle.MODE_GRADIENT,
                                                       W.MG_ALPHA, oracle.TH_RELMAX, 0, oo)
                assert sts[g].K == so.K
            else:
                xo, so, dom = oracle.local_then_global(Ah, w.b[g], w.x0[g], oracle.MODE_RESIDUAL,
                                                       W.MG_EPS, oracle.TH_PAPER, W.MG_E_MAX, oo)
                assert abs(sts[g].K - so.K) <= 2
            assert abs(sts[g].its_local - so.its_local) <= 1
            say(f"  g={g} K={sts[g].K} its={sts[g].its_local}+{sts[g].its_global} "
                f"(oracle {so.K}, {so.its_local}+{so.its_global})")


@pytest.mark.parametrize("name,dims", [("5pt", (97, 83, 1)), ("9pt", (91, 80, 1))])
def test_batched_systems_above_the_lds_size(name, dims):
    """Systems larger than the LDS-resident PCG takes (7168 cells) run the
    global-memory PCG of the same kernel: same checks against the oracle."""
    G = 2
    say("batched large", name, dims)
    A, Ahs, b, x0 = make_batch(name, G, dims)
    assert A.n > 7168
    x = dev(x0)
    sts = lcs.solve_local_then_global_batched(A, dev(b), x, "residual", "relmax", 1e-3, 1,
                                              lcs.Options(eps=1e-10))
    xg = host(x)
    for g in range(G):
        xo, so, dom = oracle.local_then_global(Ahs[g], b[g], x0[g], oracle.MODE_RESIDUAL, 1e-3,
                                               oracle.TH_RELMAX, 1, oracle.Options(eps=1e-10))
        assert sts[g].K == so.K and abs(sts[g].its_local - so.its_local) <= 1
        nb = np.linalg.norm(b[g])
        assert np.linalg.norm(oracle.residual(Ahs[g], b[g], xg[g])) <= 1.0001e-10 * nb
    xs = dev(x0)
    stg = lcs.solve_global_batched(A, dev(b), xs, lcs.Options(eps=1e-10))
    for g in range(G):
        xo, so = oracle.solve_global(Ahs[g], b[g], x0[g], oracle.Options(eps=1e-10))
        assert abs(stg[g].its_global - so.its_global) <= 1
