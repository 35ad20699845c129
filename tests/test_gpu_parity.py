"""GPU parity: the HIP path through the C ABI vs the CPU oracle.

Both sides read the same input bytes (seeded generators).  Integer and set
results (local domain, stamps, restricted CSR) and every per-row FMA-chain
result (residual, gradient, Gauss-Seidel sweeps) must match bit for bit.
Iterative results are compared (a) at equal iteration counts (trajectory
parity: only the dot-product summation order differs) and (b) after
convergence, against the criterion recomputed by the oracle.
"""
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
PC = {"jacobi": oracle.PC_JACOBI, "rbsgs": oracle.PC_SGS, "none": oracle.PC_NONE}


def say(*a):
    print("[case]", *a, flush=True)


def dev(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype).to(DEV)


def host(t):
    return t.detach().cpu().numpy()


# ragged grids: sizes that are not multiples of the 256-row blocks or the
# 2048-stamp compaction tiles, spanning several of each.  nx odd runs the
# scalar (one cell per thread) kernels; nx a multiple of 4 runs the vector
# strips (2 FP64 / 4 FP32 cells per thread) with ragged ny, nz.
CASES = {
    "5pt": (W.KIND_5PT, (93, 71, 1)),
    "9pt": (W.KIND_9PT, (83, 67, 1)),
    "7pt": (W.KIND_7PT, (23, 19, 17)),
    "5pt_v": (W.KIND_5PT, (96, 71, 1)),
    "9pt_v": (W.KIND_9PT, (84, 67, 1)),
    "7pt_v": (W.KIND_7PT, (24, 19, 17)),
    # rows of whole 8-cell words: the word-wise expansion round
    "9pt_w": (W.KIND_9PT, (88, 61, 1)),
}


def make_case(name, seed=0, dt=4.0):
    kind, (nx, ny, nz) = CASES[name]
    if kind == W.KIND_5PT:
        logk = W.lognormal_logk((ny, nx), 1.0, 100 + seed)
        coef = W.assemble_5pt(logk, 1.0 / dt)
    elif kind == W.KIND_9PT:
        coef = W.assemble_9pt(nx, ny, 1.0 / dt, 100.0, 30.0)
    else:
        logk = W.lognormal_logk((nz, ny, nx), 1.0, 100 + seed)
        coef = W.assemble_7pt(logk, 1.0 / dt)
    n = nx * ny * nz
    rng = np.random.default_rng(seed)
    # previous state x_true (background + hot box); x0 differs from it only on
    # a central box, so r^(0) = A (x_true - x0) is localized
    x_true = np.full(n, 0.1)
    g = x_true.reshape(nz, ny, nx)
    g[nz // 3: nz // 3 + max(1, nz // 3), ny // 3: ny // 3 + 9, nx // 4: nx // 4 + 11] = 1.0
    f = 0.62 if nz == 1 else 0.72
    sl = tuple(slice(int(m * (1 - f) / 2), int(m * (1 - f) / 2) + max(1, int(m * f)))
               for m in (nz, ny, nx))
    Ah = oracle.csr_from_stencil(kind, nx, ny, nz, coef)
    b = oracle.spmv(Ah, x_true)
    x0 = x_true.copy()
    box = x0.reshape(nz, ny, nx)[sl]
    x0.reshape(nz, ny, nx)[sl] = box * (1.0 + 0.3 * rng.random(box.shape))
    A = lcs.matrix_from_numpy(kind, nx, ny, nz, coef, DEV)
    return kind, (nx, ny, nz), coef, Ah, A, b, x0


# Tilings of the stencil kernels: the automatic one (the flat walk at these
# sizes), and 5-row (3-D: 5-plane) marching tiles (a partial last tile, rows
# carried in registers) with non-temporal coefficient loads.
TILINGS = {"auto": (0, -1), "rows5_nt": (5, 1)}


@pytest.fixture(scope="module", params=list(TILINGS))
def ctx(request):
    c = lcs.Context()
    lcs.set_tiling(*TILINGS[request.param], ctx=c)
    return c


# ----------------------------------------------------------------------------
# per-row kernels: bit-exact
# ----------------------------------------------------------------------------
@pytest.mark.parametrize("name", list(CASES))
def test_residual_and_gradient_bitexact(name, ctx):
    kind, dims, coef, Ah, A, b, x0 = make_case(name)
    say("residual/gradient", name, dims)
    r = host(lcs.residual(A, dev(b), dev(x0), ctx=ctx))
    assert np.array_equal(r, oracle.residual(Ah, b, x0))
    g = host(lcs.gradient(A, dev(x0), ctx=ctx))
    assert np.array_equal(g, oracle.gradient(Ah, x0))


@pytest.mark.parametrize("name", list(CASES))
def test_gs_sweeps_bitexact(name, ctx):
    kind, dims, coef, Ah, A, b, x0 = make_case(name)
    say("gs sweeps", name, dims)
    x = dev(x0)
    lcs.gs_sweeps(A, dev(b), x, 2, ctx=ctx)
    assert np.array_equal(host(x), oracle.gs_sweeps(Ah, b, x0, 2))


@pytest.mark.parametrize("dims", [(1008, 2001), (264, 67), (128, 64), (132, 5), (4, 9), (8, 1),
                                  (256, 2)])
def test_nine_point_paired_sweeps_bitexact(dims, ctx):
    """The nine-point sweep on strips of two cells runs colours (0, 1) and
    (2, 3) as two row-parity passes, each wave owning 63 strips plus one halo
    strip: grids of several strips per row, an odd number of rows per tile
    (1008 x 2001), a single strip, a single row and two rows give the
    oracle's colour-ordered sweeps bit for bit, also with a nonzero
    background, and inside Algorithm 1."""
    nx, ny = dims
    coef = W.assemble_9pt(nx, ny, 0.25, 100.0, 30.0)
    Ah = oracle.csr_from_stencil(W.KIND_9PT, nx, ny, 1, coef)
    rng = np.random.default_rng(nx + ny)
    b = rng.random(nx * ny)
    x0 = rng.random(nx * ny) - 0.5
    A = lcs.matrix_from_numpy(W.KIND_9PT, nx, ny, 1, coef, DEV)
    say("paired sweeps", dims)
    for sweeps in (1, 2):
        x = dev(x0)
        lcs.gs_sweeps(A, dev(b), x, sweeps, ctx=ctx)
        assert np.array_equal(host(x), oracle.gs_sweeps(Ah, b, x0, sweeps)), sweeps
    if nx * ny >= 64:
        # steps 3-7 of Algorithm 1: two local PCG iterations, then the sweep
        d = oracle.build_local_domain(Ah, b, x0, oracle.MODE_RESIDUAL, 1e-2, oracle.TH_RELMAX, 1)
        x = dev(x0)
        lcs.solve_local(A, dev(b), x, torch.as_tensor(d.idx).to(DEV),
                        lcs.Options(eps=1e-10, max_iter=2, check_every=1), ctx=ctx)
        xo, _ = oracle.solve_local(Ah, b, x0, d.idx, oracle.Options(eps=1e-10, max_iter=2))
        assert np.linalg.norm(host(x) - xo) <= 1e-12 * np.linalg.norm(xo)


@pytest.mark.parametrize("dims", [(1008, 2001), (264, 67), (252, 37), (128, 64), (132, 5), (4, 9),
                                  (8, 1), (256, 2)])
def test_nine_point_sweep_forms_the_criterion(dims, ctx):
    """The last pass of Algorithm 1's nine-point sweep also forms the
    criterion of step 8 (each wave owning 62 strips, with the rows next to
    its tile updated again where they have the pass's parity): on an empty
    domain, solve_local returns the oracle's colour-ordered sweeps bit for
    bit, and the relative residual it reports is the oracle's residual of
    that x up to the summation order."""
    nx, ny = dims
    coef = W.assemble_9pt(nx, ny, 0.25, 100.0, 30.0)
    Ah = oracle.csr_from_stencil(W.KIND_9PT, nx, ny, 1, coef)
    rng = np.random.default_rng(3 * nx + ny)
    b = rng.random(nx * ny)
    x0 = rng.random(nx * ny) - 0.5
    A = lcs.matrix_from_numpy(W.KIND_9PT, nx, ny, 1, coef, DEV)
    empty = torch.empty(0, dtype=torch.int32, device=DEV)
    for sweeps in (1, 2):
        say("sweep + criterion", dims, sweeps)
        x = dev(x0)
        st = lcs.solve_local(A, dev(b), x, empty, lcs.Options(eps=1e-10, n_smooth=sweeps), ctx=ctx)
        xs = oracle.gs_sweeps(Ah, b, x0, sweeps)
        assert np.array_equal(host(x), xs), sweeps
        rel = np.linalg.norm(oracle.residual(Ah, b, xs)) / np.linalg.norm(b)
        assert abs(st.relres_final - rel) <= 1e-13 * rel, (st.relres_final, rel)


@pytest.mark.parametrize("dims", [(1008, 2001), (2048, 1030)])
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_one_pass_sweep_from_the_score_copy(dims, prec):
    """Algorithm 1 on grids where the nine-point sweep runs in one pass: the
    score pass copies x^(0) into the sweep's second buffer, step 6 keeps the
    copy equal to x, and the single sweep reads it and writes x (no copy
    back).  x^(0) differs from the solution on a box, which the domain
    covers, so the local solve and the sweep meet the criterion.  The result
    equals solve_local's on the same domain (the sweep from x with a copy
    back) bit for bit, and the oracle's within the criterion."""
    nx, ny = dims
    coef = W.assemble_9pt(nx, ny, 0.25, 100.0, 30.0)
    Ah = oracle.csr_from_stencil(W.KIND_9PT, nx, ny, 1, coef)
    rng = np.random.default_rng(nx + 7 * ny)
    x_true = 0.1 + 0.01 * rng.random(nx * ny)
    b = oracle.spmv(Ah, x_true)
    x0 = x_true.copy()
    g = x0.reshape(ny, nx)
    g[ny // 3: ny // 3 + 40, nx // 2: nx // 2 + 50] *= 1.0 + 0.3 * rng.random((40, 50))
    A = lcs.matrix_from_numpy(W.KIND_9PT, nx, ny, 1, coef, DEV)
    opts = lcs.Options(eps=1e-10, precision=prec)
    say("one-pass sweep from the score copy", dims, prec)
    x = dev(x0)
    st = lcs.solve_local_then_global(A, dev(b), x, "residual", "relmax", 1e-12, 1, opts,
                                     ctx=lcs.Context())
    assert st.its_global == 0 and st.relres_final <= 1e-10, (st.its_global, st.relres_final)
    c2 = lcs.Context()
    idx, _, _ = lcs.build_local_domain(A, dev(b), dev(x0), "residual", "relmax", 1e-12, 1, ctx=c2)
    assert idx.numel() == st.K > 2000
    x2 = dev(x0)
    st2 = lcs.solve_local(A, dev(b), x2, idx, opts, ctx=c2)
    assert np.array_equal(host(x), host(x2))
    assert abs(st.relres_final - st2.relres_final) <= 1e-13 * st2.relres_final
    xo, so = oracle.solve_local(Ah, b, x0, host(idx), oracle.Options(eps=1e-10))
    rel = np.linalg.norm(host(x) - xo) / np.linalg.norm(xo)
    assert rel <= 1e-9, rel


@pytest.mark.parametrize("name", list(CASES))
def test_spmv_fp64(name, ctx):
    kind, dims, coef, Ah, A, b, x0 = make_case(name)
    say("spmv", name, dims)
    y = torch.empty(A.n, dtype=torch.float64, device=DEV)
    lcs.spmv(A, dev(x0), y, ctx=ctx)
    assert np.array_equal(host(y), oracle.spmv(Ah, x0))


@pytest.mark.parametrize("name", list(CASES))
def test_spmv_fp32(name, ctx):
    """FP32 SpMV (the inner operator of the mixed path): within the FP32
    rounding bound of a 9-term fused sum, nb * u32 * sum_j |a_ij x_j|, of the
    FP64 product of the same FP32-rounded inputs."""
    kind, dims, coef, Ah, A, b, x0 = make_case(name)
    say("spmv fp32", name, dims)
    A.coef32 = lcs.cast_coef(A, ctx=ctx)
    x32 = dev(x0, torch.float32)
    y = torch.empty(A.n, dtype=torch.float32, device=DEV)
    lcs.spmv(A, x32, y, ctx=ctx)
    c32 = host(A.coef32).astype(np.float64)
    np.testing.assert_array_equal(c32, coef.astype(np.float32).astype(np.float64))
    A32h = oracle.csr_from_stencil(kind, *dims, c32)
    xr = host(x32).astype(np.float64)
    ref = oracle.spmv(A32h, xr)
    absA = oracle.CSR(A32h.n, A32h.rp, A32h.col, np.abs(A32h.val))
    bound = 9 * 2.0 ** -24 * oracle.spmv(absA, np.abs(xr)) + 1e-30
    assert np.all(np.abs(host(y).astype(np.float64) - ref) <= bound)


# ----------------------------------------------------------------------------
# local domain (Algorithms 2 and 3): bit-exact sets and stamps
# ----------------------------------------------------------------------------
@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("mode,thresh,theta,e_max", [
    ("residual", "relmax", 1e-3, 0), ("residual", "relmax", 1e-3, 1),
    ("residual", "relmax", 1e-5, 3), ("residual", "abs", 1e-7, 2),
    ("gradient", "relmax", 1e-2, 0), ("gradient", "relmax", 1e-4, 2),
    ("residual", "relmax", 1.0, 1), ("gradient", "relmax", 0.0, 0),
])
def test_local_domain_bitexact(name, mode, thresh, theta, e_max, ctx):
    kind, dims, coef, Ah, A, b, x0 = make_case(name)
    say("domain", name, dims, mode, thresh, theta, e_max)
    idx, mask, st = lcs.build_local_domain(A, dev(b), dev(x0), mode, thresh, theta, e_max,
                                           want_mask=True, ctx=ctx)
    om = {"residual": oracle.MODE_RESIDUAL, "gradient": oracle.MODE_GRADIENT}[mode]
    ot = {"relmax": oracle.TH_RELMAX, "abs": oracle.TH_ABS}[thresh]
    d = oracle.build_local_domain(Ah, b, x0, om, theta, ot, e_max)
    assert st.K == d.K
    assert st.tau == d.tau
    assert st.e_rounds == d.rounds
    assert np.array_equal(host(idx), d.idx)
    assert np.array_equal(host(mask), d.mask)


@pytest.mark.parametrize("name", ["5pt", "7pt", "5pt_v"])
def test_local_domain_paper_threshold(name, ctx):
    """tau = eps ||b|| / sqrt(N): ||b||^2 is summed in a different order on
    the two sides; a sum of N positive terms in any order is within (N-1)u
    relative of the exact one, so the two thresholds agree to about N*u and
    only points within that band of tau may be classified differently."""
    kind, dims, coef, Ah, A, b, x0 = make_case(name)
    say("domain paper threshold", name, dims)
    idx, mask, st = lcs.build_local_domain(A, dev(b), dev(x0), "residual", "paper", 1e-8, 1,
                                           want_mask=True, ctx=ctx)
    d = oracle.build_local_domain(Ah, b, x0, oracle.MODE_RESIDUAL, 1e-8, oracle.TH_PAPER, 1)
    band = A.n * np.finfo(np.float64).eps * d.tau
    assert abs(st.tau - d.tau) <= band
    diff = np.nonzero(host(mask) != d.mask)[0]
    r = d.score
    for i in diff:   # only near-ties of the threshold may differ
        assert abs(abs(r[i]) - d.tau) <= 2 * band


def test_empty_and_full_domains(ctx):
    kind, dims, coef, Ah, A, b, x0 = make_case("5pt")
    say("empty/full domains")
    xs = oracle.spmv(Ah, x0)   # b = A x0 exactly: r = 0 up to rounding
    idx, _, st = lcs.build_local_domain(A, dev(np.zeros(A.n)), dev(np.zeros(A.n)), "residual",
                                        "relmax", 1e-3, 2, ctx=ctx)
    assert st.K == 0 and idx.numel() == 0
    idx, _, st = lcs.build_local_domain(A, dev(b), dev(x0), "residual", "abs", 0.0, 0, ctx=ctx)
    d = oracle.build_local_domain(Ah, b, x0, oracle.MODE_RESIDUAL, 0.0, oracle.TH_ABS, 0)
    assert st.K == d.K and np.array_equal(host(idx), d.idx)
    del xs


@pytest.mark.parametrize("mode,thresh,theta", [("residual", "paper", 1e-10),
                                               ("gradient", "relmax", 1e-4)])
def test_converged_x0_returned_unchanged(mode, thresh, theta, ctx):
    """x0 meeting the criterion: the solution is x0 itself, bit for bit, with
    no local or global iteration (as the oracle and the global PCG)."""
    kind, dims, coef, Ah, A, b, x0 = make_case("5pt")
    say("converged x0", mode)
    nb = np.linalg.norm(b)
    xs = oracle.pcg(Ah, b, x0, oracle.PC_JACOBI, 1e-13 * nb, 5000)[0]
    xo, so, dom = oracle.local_then_global(Ah, b, xs, oracle.MODE_RESIDUAL, 1e-10,
                                           oracle.TH_PAPER, 1, oracle.Options(eps=1e-10))
    assert dom.K == 0 and np.array_equal(xo, xs)
    x = dev(xs)
    st = lcs.solve_local_then_global(A, dev(b), x, mode, thresh, theta, 1, lcs.Options(eps=1e-10),
                                     ctx=ctx)
    assert st.K == 0 and st.its_local == 0 and st.its_global == 0
    assert np.array_equal(host(x), xs)
    assert st.relres_final <= 1e-10


# ----------------------------------------------------------------------------
# restricted system (eq. BEFC): bit-exact CSR
# ----------------------------------------------------------------------------
@pytest.mark.parametrize("name", list(CASES))
def test_gather_restricted_bitexact(name, ctx):
    kind, dims, coef, Ah, A, b, x0 = make_case(name)
    say("gather", name, dims)
    d = oracle.build_local_domain(Ah, b, x0, oracle.MODE_RESIDUAL, 1e-4, oracle.TH_RELMAX, 1)
    assert d.K > 2048   # spans several compaction tiles
    rp, col, val = lcs.gather_restricted(A, dev(d.idx, torch.int32), ctx=ctx)
    B = oracle.restricted(Ah, d.idx)
    assert np.array_equal(host(rp).astype(np.int64), B.rp)
    assert np.array_equal(host(col), B.col)
    assert np.array_equal(host(val), B.val)


def test_gather_rejects_bad_domain(ctx):
    kind, dims, coef, Ah, A, b, x0 = make_case("5pt")
    say("gather rejects bad idx")
    bad = dev(np.array([3, 2, 7], np.int32), torch.int32)          # not ascending
    with pytest.raises(lcs.LcsError) as e:
        lcs.gather_restricted(A, bad, ctx=ctx)
    assert e.value.status == lcs.EINVAL
    bad = dev(np.array([1, A.n + 5], np.int32), torch.int32)       # out of range
    with pytest.raises(lcs.LcsError):
        lcs.gather_restricted(A, bad, ctx=ctx)


# ----------------------------------------------------------------------------
# PCG: trajectory parity at equal iteration counts, converged parity
# ----------------------------------------------------------------------------
@pytest.mark.parametrize("name,pc", [("5pt", "jacobi"), ("9pt", "jacobi"), ("7pt", "jacobi"),
                                     ("5pt", "rbsgs"), ("7pt", "rbsgs"), ("5pt", "none"),
                                     ("5pt_v", "jacobi"), ("9pt_v", "jacobi"), ("7pt_v", "rbsgs"),
                                     ("9pt", "rbsgs"), ("9pt_v", "rbsgs")])
def test_global_pcg_parity(name, pc, ctx):
    kind, dims, coef, Ah, A, b, x0 = make_case(name)
    say("global pcg", name, dims, pc)
    oo = oracle.Options(eps=1e-10, pc=PC[pc])
    xo, so = oracle.solve_global(Ah, b, x0, oo)
    assert so.status == oracle.OK
    x = dev(x0)
    st = lcs.solve_global(A, dev(b), x, lcs.Options(eps=1e-10, precond=pc), ctx=ctx)
    xg = host(x)
    nb = np.linalg.norm(b)
    assert np.linalg.norm(oracle.residual(Ah, b, xg)) <= 1.0001e-10 * nb
    assert abs(st.its_global - so.its_global) <= 1
    # trajectory parity: stop both at the same iteration count.  CG amplifies
    # rounding differences as iterations go on (loss of orthogonality), so
    # compare within the first 20 iterations, where a wrong index, sign or
    # coefficient would still show at O(1).
    m = max(min(so.its_global // 2, 20), 1)
    xo_m, sto, it_o, _ = oracle.pcg(Ah, b, x0, PC[pc], 0.0, m)
    xm = dev(x0)
    with pytest.raises(lcs.LcsError) as e:
        lcs.solve_global(A, dev(b), xm, lcs.Options(eps=1e-30, precond=pc, max_iter=m,
                                                    max_outer=0), ctx=ctx)
    assert e.value.status == lcs.ENOCONV
    rel = np.linalg.norm(host(xm) - xo_m) / np.linalg.norm(xo_m)
    assert rel <= 1e-10, rel


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("mode,thresh,theta", [("residual", "relmax", 1e-3),
                                               ("residual", "relmax", 0.3),
                                               ("residual", "paper", 1e-10),
                                               ("gradient", "relmax", 1e-4)])
def test_local_then_global_parity(name, mode, thresh, theta, ctx):
    kind, dims, coef, Ah, A, b, x0 = make_case(name)
    say("local_then_global", name, dims, mode, thresh, theta)
    om = {"residual": oracle.MODE_RESIDUAL, "gradient": oracle.MODE_GRADIENT}[mode]
    ot = {"relmax": oracle.TH_RELMAX, "paper": oracle.TH_PAPER}[thresh]
    xo, so, dom = oracle.local_then_global(Ah, b, x0, om, theta, ot, 1, oracle.Options(eps=1e-10))
    x = dev(x0)
    st = lcs.solve_local_then_global(A, dev(b), x, mode, thresh, theta, 1, lcs.Options(eps=1e-10),
                                     ctx=ctx)
    xg = host(x)
    nb = np.linalg.norm(b)
    if thresh != "paper":
        assert st.K == so.K
    else:
        assert abs(st.K - so.K) <= 2
    assert abs(st.its_local - so.its_local) <= 1
    assert np.linalg.norm(oracle.residual(Ah, b, xg)) <= 1.0001e-10 * nb
    xd = oracle.pcg(Ah, b, xo, oracle.PC_JACOBI, 1e-14 * nb, 5000)[0]   # tight reference
    err_g = np.linalg.norm(xg - xd) / np.linalg.norm(xd)
    err_o = np.linalg.norm(xo - xd) / np.linalg.norm(xd)
    say(f"  K={st.K} its_local={st.its_local} its_global={st.its_global} err_gpu={err_g:.2e} "
        f"err_oracle={err_o:.2e}")
    assert err_g <= max(10 * err_o, 1e-10)


@pytest.mark.parametrize("name", ["9pt", "9pt_v"])
@pytest.mark.parametrize("mode,theta", [("residual", 1e-3), ("gradient", 1e-4)])
def test_local_then_global_nine_point_sgs(name, mode, theta, ctx):
    """Algorithm 1 on the nine-point stencil with the four-colour symmetric
    Gauss-Seidel preconditioner for the local and the global PCG."""
    kind, dims, coef, Ah, A, b, x0 = make_case(name)
    say("local_then_global sgs9", name, dims, mode)
    om = {"residual": oracle.MODE_RESIDUAL, "gradient": oracle.MODE_GRADIENT}[mode]
    oo = oracle.Options(eps=1e-10, pc=oracle.PC_SGS)
    xo, so, dom = oracle.local_then_global(Ah, b, x0, om, theta, oracle.TH_RELMAX, 1, oo)
    x = dev(x0)
    st = lcs.solve_local_then_global(A, dev(b), x, mode, "relmax", theta, 1,
                                     lcs.Options(eps=1e-10, precond="rbsgs"), ctx=ctx)
    assert st.K == so.K
    assert abs(st.its_local - so.its_local) <= 1 and abs(st.its_global - so.its_global) <= 1
    nb = np.linalg.norm(b)
    xg = host(x)
    assert np.linalg.norm(oracle.residual(Ah, b, xg)) <= 1.0001e-10 * nb
    xd = oracle.pcg(Ah, b, xo, oracle.PC_JACOBI, 1e-14 * nb, 5000)[0]
    err_g = np.linalg.norm(xg - xd) / np.linalg.norm(xd)
    err_o = np.linalg.norm(xo - xd) / np.linalg.norm(xd)
    say(f"  K={st.K} its={st.its_local}+{st.its_global} (oracle {so.its_local}+{so.its_global}) "
        f"err {err_g:.1e} / {err_o:.1e}")
    assert err_g <= max(10 * err_o, 1e-10)


@pytest.mark.parametrize("name", ["7pt", "7pt_v", "9pt_v", "5pt"])
def test_colour_blocked_restricted_system(name):
    """Under RB-SGS the local domain is reordered colour by colour before
    the gather (each half sweep reads its own colour's rows); with the
    reordering switched off B keeps the domain's ascending order.  Every
    per-row result is the same, so equal iteration counts give solutions
    that differ only by the reductions' summation order, and both follow
    the oracle's trajectory."""
    kind, dims, coef, Ah, A, b, x0 = make_case(name)
    d = oracle.build_local_domain(Ah, b, x0, oracle.MODE_RESIDUAL, 1e-3, oracle.TH_RELMAX, 1)
    assert d.K > 100
    oo = oracle.Options(eps=1e-10, max_iter=6, pc=oracle.PC_SGS)
    xo, _ = oracle.solve_local(Ah, b, x0, d.idx, oo)
    xs = []
    for on in (True, False):
        say("colour blocks", name, dims, on)
        c = lcs.Context()
        lcs.set_colour_blocking(on, ctx=c)
        x = dev(x0)
        lcs.solve_local(A, dev(b), x, dev(d.idx, torch.int32),
                        lcs.Options(eps=1e-10, max_iter=6, check_every=1, precond="rbsgs"), ctx=c)
        xs.append(host(x))
        assert np.linalg.norm(xs[-1] - xo) <= 1e-12 * np.linalg.norm(xo), on
    assert np.linalg.norm(xs[0] - xs[1]) <= 1e-13 * np.linalg.norm(xs[1])


@pytest.mark.parametrize("name", ["5pt", "5pt_v", "9pt", "9pt_v", "9pt_w"])
@pytest.mark.parametrize("prec,pc", [("mixed", "jacobi"), ("fp64", "jacobi"), ("mixed", "rbsgs")])
def test_short_column_form(name, prec, pc):
    """The restricted system's columns coded per row (fixed stencil slots,
    offsets to the rows below and above and presence bits: the default on
    the 2-D stencils) or as 32-bit indices: the same members in the same
    order, so the local solve returns the same x and iteration count bit for
    bit.  Under RB-SGS with colour blocking off, so that the domain keeps its
    grid order."""
    kind, dims, coef, Ah, A, b, x0 = make_case(name)
    d = oracle.build_local_domain(Ah, b, x0, oracle.MODE_RESIDUAL, 1e-3, oracle.TH_RELMAX, 1)
    assert d.K > 100
    xs, its = [], []
    for on in (True, False):
        say("short columns", name, dims, prec, pc, on)
        c = lcs.Context()
        lcs.set_short_columns(on, ctx=c)
        lcs.set_colour_blocking(False, ctx=c)
        x = dev(x0)
        st = lcs.solve_local(A, dev(b), x, dev(d.idx, torch.int32),
                             lcs.Options(eps=1e-10, precision=prec, precond=pc), ctx=c)
        xs.append(host(x))
        its.append(st.its_local)
    assert its[0] == its[1] > 0
    assert np.array_equal(xs[0], xs[1])


@pytest.mark.parametrize("name", ["5pt", "5pt_v", "7pt", "7pt_v"])
@pytest.mark.parametrize("prec", ["mixed", "fp64"])
def test_red_black_row_codes(name, prec):
    """RB-SGS with the restricted rows blocked by colour: on the five- and
    seven-point stencils each row's columns are coded from its position in
    the other colour's block (the default) or stored as 32-bit indices.  The
    same members in the same order, so the local solve returns the same x
    and iteration count bit for bit, and follows the oracle."""
    kind, dims, coef, Ah, A, b, x0 = make_case(name)
    d = oracle.build_local_domain(Ah, b, x0, oracle.MODE_RESIDUAL, 1e-3, oracle.TH_RELMAX, 1)
    assert d.K > 100
    xs, its = [], []
    for on in (True, False):
        say("red-black row codes", name, dims, prec, on)
        c = lcs.Context()
        lcs.set_short_columns(on, ctx=c)
        x = dev(x0)
        st = lcs.solve_local(A, dev(b), x, dev(d.idx, torch.int32),
                             lcs.Options(eps=1e-10, precision=prec, precond="rbsgs"), ctx=c)
        xs.append(host(x))
        its.append(st.its_local)
    assert its[0] == its[1] > 0
    assert np.array_equal(xs[0], xs[1])
    xo, _ = oracle.solve_local(Ah, b, x0, d.idx, oracle.Options(eps=1e-10, pc=oracle.PC_SGS))
    rel = np.linalg.norm(xs[0] - xo) / np.linalg.norm(xo)
    assert rel <= 1e-9, rel


@pytest.mark.parametrize("kind,dims", [(W.KIND_5PT, (131068, 3, 1)), (W.KIND_7PT, (362, 362, 3)),
                                       (W.KIND_7PT, (363, 362, 3))])
def test_red_black_row_codes_at_the_limit(kind, dims):
    """Whole-grid domains under RB-SGS on grids as wide as the red-black
    codes' 16-bit distances allow (half a row of 131068 cells; half a plane
    of 362 x 362) and one wider plane (363 x 362: 32-bit indices).  The two
    forms agree bit for bit, and both follow the oracle's trajectory."""
    nx, ny, nz = dims
    dt = 4.0
    if kind == W.KIND_5PT:
        coef = W.assemble_5pt(W.lognormal_logk((ny, nx), 1.0, 11), 1.0 / dt)
    else:
        coef = W.assemble_7pt(W.lognormal_logk((nz, ny, nx), 1.0, 11), 1.0 / dt)
    n = nx * ny * nz
    rng = np.random.default_rng(13)
    Ah = oracle.csr_from_stencil(kind, nx, ny, nz, coef)
    b = oracle.spmv(Ah, rng.random(n))
    x0 = np.zeros(n)
    idx = np.arange(n, dtype=np.int32)
    xo, so = oracle.solve_local(Ah, b, x0, idx,
                                oracle.Options(eps=1e-10, max_iter=6, n_smooth=1, pc=oracle.PC_SGS))
    A = lcs.matrix_from_numpy(kind, nx, ny, nz, coef, DEV)
    xs = []
    for on in (True, False):
        say("red-black row codes at the limit", kind, dims, on)
        c = lcs.Context()
        lcs.set_short_columns(on, ctx=c)
        x = dev(x0)
        st = lcs.solve_local(A, dev(b), x, dev(idx, torch.int32),
                             lcs.Options(eps=1e-10, max_iter=6, n_smooth=1, check_every=1,
                                         precond="rbsgs"), ctx=c)
        assert st.its_local == so.its_local == 6
        xs.append(host(x))
        rel = np.linalg.norm(xs[-1] - xo) / np.linalg.norm(xo)
        assert rel <= 1e-12, (on, rel)
    assert np.array_equal(xs[0], xs[1])


@pytest.mark.parametrize("kind,nx", [(W.KIND_5PT, 32767), (W.KIND_9PT, 32766),
                                     (W.KIND_9PT, 32767)])
def test_short_columns_at_the_offset_limit(kind, nx):
    """Whole-grid domains on grids as wide as the row codes' 16-bit offsets
    allow (the five-point stencil's rows below and above 32767 rows away at
    nx = 32767; the nine-point stencil's reach nx + 1 = 32767 at nx = 32766)
    and one wider (nx = 32767 on the nine-point stencil: 32-bit indices).
    The two forms agree bit for bit, and both follow the oracle's
    trajectory."""
    ny, dt = 5, 4.0
    if kind == W.KIND_5PT:
        coef = W.assemble_5pt(W.lognormal_logk((ny, nx), 1.0, 7), 1.0 / dt)
    else:
        coef = W.assemble_9pt(nx, ny, 1.0 / dt, 100.0, 30.0)
    n = nx * ny
    rng = np.random.default_rng(3)
    Ah = oracle.csr_from_stencil(kind, nx, ny, 1, coef)
    b = oracle.spmv(Ah, rng.random(n))
    x0 = np.zeros(n)
    idx = np.arange(n, dtype=np.int32)
    oo = oracle.Options(eps=1e-10, max_iter=6, n_smooth=1, pc=oracle.PC_JACOBI)
    xo, so = oracle.solve_local(Ah, b, x0, idx, oo)
    A = lcs.matrix_from_numpy(kind, nx, ny, 1, coef, DEV)
    xs = []
    for on in (True, False):
        say("short columns at the limit", kind, nx, ny, on)
        c = lcs.Context()
        lcs.set_short_columns(on, ctx=c)
        x = dev(x0)
        st = lcs.solve_local(A, dev(b), x, dev(idx, torch.int32),
                             lcs.Options(eps=1e-10, max_iter=6, n_smooth=1, check_every=1),
                             ctx=c)
        assert st.its_local == so.its_local == 6
        xs.append(host(x))
        rel = np.linalg.norm(xs[-1] - xo) / np.linalg.norm(xo)
        assert rel <= 1e-12, (on, rel)
    assert np.array_equal(xs[0], xs[1])


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("pc", ["jacobi", "rbsgs"])
def test_solve_local_trajectory_parity(name, pc, ctx):
    """Local PCG on B stopped at equal iteration counts, then assembly and one
    GS sweep: rounding-level agreement with the oracle.  With rbsgs the
    restricted rows keep the colours of their cells (four on the nine-point
    stencil)."""
    kind, dims, coef, Ah, A, b, x0 = make_case(name)
    say("solve_local trajectory", name, dims, pc)
    d = oracle.build_local_domain(Ah, b, x0, oracle.MODE_RESIDUAL, 1e-4, oracle.TH_RELMAX, 1)
    oo = oracle.Options(eps=1e-10, max_iter=7, n_smooth=1, pc=PC[pc])
    xo, so = oracle.solve_local(Ah, b, x0, d.idx, oo)
    x = dev(x0)
    st = lcs.solve_local(A, dev(b), x, dev(d.idx, torch.int32),
                         lcs.Options(eps=1e-10, max_iter=7, n_smooth=1, precond=pc), ctx=ctx)
    assert st.its_local == so.its_local == 7
    rel = np.linalg.norm(host(x) - xo) / np.linalg.norm(xo)
    assert rel <= 1e-12, rel


# ----------------------------------------------------------------------------
# mixed precision: FP32 inner sweeps + FP64 refinement
# ----------------------------------------------------------------------------
@pytest.mark.parametrize("name,pc", [("5pt", "jacobi"), ("9pt", "jacobi"), ("7pt", "rbsgs"),
                                     ("5pt_v", "jacobi"), ("9pt_v", "jacobi"), ("7pt_v", "rbsgs"),
                                     ("9pt", "rbsgs")])
def test_mixed_precision_refinement(name, pc, ctx):
    kind, dims, coef, Ah, A, b, x0 = make_case(name)
    say("mixed", name, dims, pc)
    nb = np.linalg.norm(b)
    xd = oracle.pcg(Ah, b, x0, oracle.PC_JACOBI, 1e-14 * nb, 5000)[0]
    xo, so = oracle.solve_global(Ah, b, x0, oracle.Options(eps=1e-10, pc=PC[pc]))
    err_o = np.linalg.norm(xo - xd) / np.linalg.norm(xd)
    for call in ("global", "local"):
        x = dev(x0)
        o = lcs.Options(eps=1e-10, precond=pc, precision="mixed")
        if call == "global":
            st = lcs.solve_global(A, dev(b), x, o, ctx=ctx)
        else:
            st = lcs.solve_local_then_global(A, dev(b), x, "residual", "relmax", 1e-3, 1, o, ctx=ctx)
        xg = host(x)
        assert np.linalg.norm(oracle.residual(Ah, b, xg)) <= 1.0001e-10 * nb
        err = np.linalg.norm(xg - xd) / np.linalg.norm(xd)
        say(f"  {call}: outer={st.n_outer} its={st.its_local}+{st.its_global} err={err:.2e} "
            f"fp64 oracle err={err_o:.2e}")
        assert err <= max(10 * err_o, 1e-9)


# ----------------------------------------------------------------------------
# determinism and error paths
# ----------------------------------------------------------------------------
def test_run_twice_bitwise(ctx):
    kind, dims, coef, Ah, A, b, x0 = make_case("5pt")
    say("run twice")
    out = []
    for _ in range(2):
        x = dev(x0)
        lcs.solve_local_then_global(A, dev(b), x, "residual", "relmax", 1e-3, 1, ctx=ctx)
        out.append(host(x))
    assert np.array_equal(out[0], out[1])


def test_argument_errors(ctx):
    kind, dims, coef, Ah, A, b, x0 = make_case("9pt")
    say("argument errors")
    with pytest.raises(lcs.LcsError):
        lcs.build_local_domain(A, dev(b), dev(x0), "gradient", "paper", 1e-3, 0, ctx=ctx)
    with pytest.raises(lcs.LcsError):
        lcs.build_local_domain(A, dev(b), dev(x0), "residual", "relmax", 1e-3, 300, ctx=ctx)
    with pytest.raises(lcs.LcsError) as e:
        lcs.set_tiling(4, 2, ctx=lcs.Context())
    assert e.value.status == lcs.EINVAL


@pytest.mark.parametrize("name", ["5pt_v", "9pt_v", "7pt_v"])
@pytest.mark.parametrize("rows,nt", [(-1, -1), (3, 0), (7, 1), (200, 1)])
def test_walks_agree_bitwise(name, rows, nt):
    """Every walk of the stencil kernels (flat; marching up rows or planes
    with and without the non-temporal hints; tiles taller than the grid) gives
    the oracle's per-row results bit for bit, and Algorithm 1 meets the
    criterion."""
    kind, dims, coef, Ah, A, b, x0 = make_case(name)
    say("walk", name, rows, nt)
    c = lcs.Context()
    lcs.set_tiling(rows, nt, ctx=c)
    r = host(lcs.residual(A, dev(b), dev(x0), ctx=c))
    assert np.array_equal(r, oracle.residual(Ah, b, x0))
    x = dev(x0)
    lcs.gs_sweeps(A, dev(b), x, 1, ctx=c)
    assert np.array_equal(host(x), oracle.gs_sweeps(Ah, b, x0, 1))
    x = dev(x0)
    lcs.solve_local_then_global(A, dev(b), x, "residual", "relmax", 1e-3, 1, ctx=c)
    assert np.linalg.norm(oracle.residual(Ah, b, host(x))) <= 1.0001e-10 * np.linalg.norm(b)


def test_nonfinite_input_reported(ctx):
    kind, dims, coef, Ah, A, b, x0 = make_case("5pt")
    say("nonfinite")
    bb = b.copy()
    bb[17] = np.nan
    with pytest.raises(lcs.LcsError) as e:
        lcs.solve_global(A, dev(bb), dev(x0), ctx=ctx)
    assert e.value.status == lcs.ENONFINITE


def test_breakdown_on_indefinite_operator(ctx):
    kind, dims, coef, Ah, A, b, x0 = make_case("5pt")
    say("breakdown")
    c = coef.copy()
    c[0] *= -1.0    # negative diagonal: not SPD
    An = lcs.matrix_from_numpy(kind, *dims, c, DEV)
    with pytest.raises(lcs.LcsError) as e:
        lcs.solve_global(An, dev(b), dev(x0), lcs.Options(precond="none"), ctx=ctx)
    assert e.value.status in (lcs.EBREAKDOWN, lcs.ENOCONV)
