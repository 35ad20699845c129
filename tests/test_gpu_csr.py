"""GPU parity on general sparse input (LCS_CSR): irregular graphs with rows
of up to 11 entries (ELL width 16), of 5 entries (width 5) and with hub rows
of 18 to 64 entries (width 64), a nine-point stencil given as CSR, and
degenerate sizes.  Per-row kernels, local domains
and the restricted system bit for bit against the oracle; global PCG and
Algorithm 1 converged and at equal iteration counts; malformed structures
rejected before any kernel reads through them."""
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


def gpu_matrix(Ah, coloured=True):
    colour = dev(Ah.colour.astype(np.uint8), torch.uint8) if coloured else None
    return lcs.CsrMatrix(dev(Ah.rp, torch.int32), dev(Ah.col, torch.int32), dev(Ah.val),
                         colour, Ah.ncolours if coloured else 0)


def irregular(nx, ny, seed, **kw):
    rp, col, val = W.irregular_spd(nx, ny, seed, **kw)
    colour, nc = W.greedy_colouring(rp, col)
    return oracle.CSR(nx * ny, rp, col, val, colour, nc), (nx, ny)


def make_case(name):
    """Oracle CSR, GPU CSR, b, x0: x_true smooth, x0 off it on a disk."""
    if name == "irr16":
        Ah, (nx, ny) = irregular(61, 47, 11)
    elif name == "hub64":   # hub rows of 18..64 entries among rows of at most 16
        Ah, (nx, ny) = irregular(61, 47, 14, hub_every=29)
    elif name == "irr8":
        Ah, (nx, ny) = irregular(53, 41, 12, p_diag=0.0, p_long=0.0)
    elif name == "grid7":   # 3-D seven-point stencil (red-black), planes stacked in y
        nx, ny, nz = 19, 17, 9
        coef = W.assemble_7pt(W.lognormal_logk((nz, ny, nx), 1.0, 13), 0.25)
        Ah = oracle.csr_from_stencil(W.KIND_7PT, nx, ny, nz, coef)
        ny *= nz
    else:   # nine-point stencil as CSR, with its four-colour grid colouring
        nx, ny = 45, 37
        coef = W.assemble_9pt(nx, ny, 0.25, 100.0, 30.0)
        Ah = oracle.csr_from_stencil(W.KIND_9PT, nx, ny, 1, coef)
    yy, xx = np.mgrid[0:ny, 0:nx]
    x_true = (0.2 + 0.1 * np.sin(xx / 7.0) * np.cos(yy / 5.0)).ravel()
    b = oracle.spmv(Ah, x_true)
    disk = ((xx - nx / 3) ** 2 + (yy - ny / 2) ** 2 < (min(nx, ny) / 6) ** 2).ravel()
    x0 = x_true.copy()
    x0[disk] += 0.5
    return Ah, gpu_matrix(Ah), b, x0


CASES = ["irr16", "irr8", "grid9", "grid7", "hub64"]   # ELL widths 16, 5, 9, 7, 64


@pytest.fixture(scope="module")
def ctx():
    return lcs.Context()


@pytest.mark.parametrize("name", CASES)
def test_csr_per_row_kernels_bitexact(name, ctx):
    Ah, A, b, x0 = make_case(name)
    say("csr per-row", name, A.n, Ah.col.size)
    assert np.array_equal(host(lcs.residual(A, dev(b), dev(x0), ctx=ctx)), oracle.residual(Ah, b, x0))
    assert np.array_equal(host(lcs.gradient(A, dev(x0), ctx=ctx)), oracle.gradient(Ah, x0))
    y = torch.empty(A.n, dtype=torch.float64, device=DEV)
    lcs.spmv(A, dev(x0), y, ctx=ctx)
    assert np.array_equal(host(y), oracle.spmv(Ah, x0))
    x = dev(x0)
    lcs.gs_sweeps(A, dev(b), x, 2, ctx=ctx)
    assert np.array_equal(host(x), oracle.gs_sweeps(Ah, b, x0, 2))


def test_csr_nine_point_equals_the_stencil_kind(ctx):
    """The nine-point stencil given as CSR and as the stencil kind: per-row
    kernels and the local domain agree bit for bit."""
    nx, ny = 45, 37
    coef = W.assemble_9pt(nx, ny, 0.25, 100.0, 30.0)
    Ah, A, b, x0 = make_case("grid9")
    S = lcs.matrix_from_numpy(W.KIND_9PT, nx, ny, 1, coef, DEV)
    say("csr vs stencil")
    assert np.array_equal(host(lcs.residual(A, dev(b), dev(x0), ctx=ctx)),
                          host(lcs.residual(S, dev(b), dev(x0), ctx=ctx)))
    ia, ma, sa = lcs.build_local_domain(A, dev(b), dev(x0), "residual", "relmax", 1e-3, 2,
                                        want_mask=True, ctx=ctx)
    ib, mb, sb = lcs.build_local_domain(S, dev(b), dev(x0), "residual", "relmax", 1e-3, 2,
                                        want_mask=True, ctx=ctx)
    assert sa.K == sb.K and np.array_equal(host(ia), host(ib)) and np.array_equal(host(ma), host(mb))


@pytest.mark.parametrize("name", CASES)
@pytest.mark.parametrize("mode,theta,e_max", [("residual", 1e-3, 2), ("residual", 0.2, 1),
                                              ("gradient", 0.3, 0)])
def test_csr_local_domain_and_gather_bitexact(name, mode, theta, e_max, ctx):
    Ah, A, b, x0 = make_case(name)
    say("csr domain", name, mode, theta, e_max)
    om = {"residual": oracle.MODE_RESIDUAL, "gradient": oracle.MODE_GRADIENT}[mode]
    d = oracle.build_local_domain(Ah, b, x0, om, theta, oracle.TH_RELMAX, e_max)
    idx, mask, st = lcs.build_local_domain(A, dev(b), dev(x0), mode, "relmax", theta, e_max,
                                           want_mask=True, ctx=ctx)
    assert 0 < d.K < Ah.n
    assert st.K == d.K and st.e_rounds == d.rounds and st.tau == d.tau
    assert np.array_equal(host(idx), d.idx) and np.array_equal(host(mask), d.mask)
    rp, col, val = lcs.gather_restricted(A, idx, ctx=ctx)
    Bo = oracle.restricted(Ah, d.idx)
    assert np.array_equal(host(rp), Bo.rp) and np.array_equal(host(col), Bo.col)
    assert np.array_equal(host(val), Bo.val)


@pytest.mark.parametrize("name,pc", [("irr16", "jacobi"), ("irr16", "rbsgs"), ("irr16", "none"),
                                     ("irr8", "jacobi"), ("irr8", "rbsgs"), ("grid9", "rbsgs"),
                                     ("grid7", "jacobi"), ("grid7", "rbsgs")])
def test_csr_global_pcg_parity(name, pc, ctx):
    Ah, A, b, x0 = make_case(name)
    say("csr global pcg", name, pc)
    xo, so = oracle.solve_global(Ah, b, x0, oracle.Options(eps=1e-10, pc=PC[pc]))
    assert so.status == oracle.OK
    x = dev(x0)
    st = lcs.solve_global(A, dev(b), x, lcs.Options(eps=1e-10, precond=pc), ctx=ctx)
    nb = np.linalg.norm(b)
    assert np.linalg.norm(oracle.residual(Ah, b, host(x))) <= 1.0001e-10 * nb
    assert abs(st.its_global - so.its_global) <= 1
    # Without the diagonal scaling, CG on these log-normal weights amplifies
    # rounding about tenfold per step (the oracle against itself, x0 perturbed
    # by 1e-15: 7e-16 after 5 steps, 2.5e-6 after 20), so "none" compares
    # after 5 steps, where a wrong index or sign would still show at O(1).
    m = max(min(so.its_global // 2, 20 if pc != "none" else 5), 1)
    xo_m = oracle.pcg(Ah, b, x0, PC[pc], 0.0, m)[0]
    xm = dev(x0)
    with pytest.raises(lcs.LcsError) as e:
        lcs.solve_global(A, dev(b), xm, lcs.Options(eps=1e-30, precond=pc, max_iter=m, max_outer=0),
                         ctx=ctx)
    assert e.value.status == lcs.ENOCONV
    rel = np.linalg.norm(host(xm) - xo_m) / np.linalg.norm(xo_m)
    assert rel <= 1e-10, rel


@pytest.mark.parametrize("name", CASES)
@pytest.mark.parametrize("coloured", [True, False])
@pytest.mark.parametrize("mode,thresh,theta", [("residual", "relmax", 1e-3),
                                               ("residual", "paper", 1e-10),
                                               ("gradient", "relmax", 1e-3)])
def test_csr_local_then_global_parity(name, coloured, mode, thresh, theta, ctx):
    """Algorithm 1; without a colouring both sides skip the smoothing step."""
    Ah, A, b, x0 = make_case(name)
    if not coloured:
        Ah = oracle.CSR(Ah.n, Ah.rp, Ah.col, Ah.val, None, 0)
        A = gpu_matrix(Ah, coloured=False)
    say("csr local_then_global", name, coloured, mode, thresh)
    om = {"residual": oracle.MODE_RESIDUAL, "gradient": oracle.MODE_GRADIENT}[mode]
    ot = {"relmax": oracle.TH_RELMAX, "paper": oracle.TH_PAPER}[thresh]
    xo, so, _ = oracle.local_then_global(Ah, b, x0, om, theta, ot, 1, oracle.Options(eps=1e-10))
    x = dev(x0)
    st = lcs.solve_local_then_global(A, dev(b), x, mode, thresh, theta, 1, lcs.Options(eps=1e-10),
                                     ctx=ctx)
    xg = host(x)
    nb = np.linalg.norm(b)
    if thresh == "paper":
        assert abs(st.K - so.K) <= 2
    else:
        assert st.K == so.K
    assert abs(st.its_local - so.its_local) <= 1
    assert np.linalg.norm(oracle.residual(Ah, b, xg)) <= 1.0001e-10 * nb
    xd = oracle.pcg(Ah, b, xo, oracle.PC_JACOBI, 1e-14 * nb, 5000)[0]
    err_g = np.linalg.norm(xg - xd) / np.linalg.norm(xd)
    err_o = np.linalg.norm(xo - xd) / np.linalg.norm(xd)
    say(f"  K={st.K} its {st.its_local}+{st.its_global} (oracle {so.its_local}+{so.its_global}) "
        f"err {err_g:.1e} / {err_o:.1e}")
    assert err_g <= max(10 * err_o, 1e-10)


@pytest.mark.parametrize("name,pc", [("irr16", "jacobi"), ("irr8", "rbsgs"), ("grid7", "rbsgs")])
def test_csr_solve_local_trajectory(name, pc, ctx):
    Ah, A, b, x0 = make_case(name)
    say("csr solve_local trajectory", name, pc)
    d = oracle.build_local_domain(Ah, b, x0, oracle.MODE_RESIDUAL, 1e-4, oracle.TH_RELMAX, 1)
    xo, so = oracle.solve_local(Ah, b, x0, d.idx, oracle.Options(eps=1e-10, max_iter=7, pc=PC[pc]))
    x = dev(x0)
    st = lcs.solve_local(A, dev(b), x, dev(d.idx, torch.int32),
                         lcs.Options(eps=1e-10, max_iter=7, precond=pc), ctx=ctx)
    assert st.its_local == so.its_local == 7
    rel = np.linalg.norm(host(x) - xo) / np.linalg.norm(xo)
    assert rel <= 1e-12, rel


@pytest.mark.parametrize("name,pc", [("irr16", "jacobi"), ("irr8", "rbsgs"), ("grid9", "jacobi"),
                                     ("grid7", "rbsgs")])
def test_csr_mixed_precision(name, pc, ctx):
    Ah, A, b, x0 = make_case(name)
    say("csr mixed", name, pc)
    nb = np.linalg.norm(b)
    xd = oracle.pcg(Ah, b, x0, oracle.PC_JACOBI, 1e-14 * nb, 5000)[0]
    xo, _ = oracle.solve_global(Ah, b, x0, oracle.Options(eps=1e-10, pc=PC[pc]))
    err_o = np.linalg.norm(xo - xd) / np.linalg.norm(xd)
    for call in ("global", "local"):
        x = dev(x0)
        o = lcs.Options(eps=1e-10, precond=pc, precision="mixed")
        if call == "global":
            lcs.solve_global(A, dev(b), x, o, ctx=ctx)
        else:
            lcs.solve_local_then_global(A, dev(b), x, "residual", "relmax", 1e-3, 1, o, ctx=ctx)
        xg = host(x)
        assert np.linalg.norm(oracle.residual(Ah, b, xg)) <= 1.0001e-10 * nb
        assert np.linalg.norm(xg - xd) / np.linalg.norm(xd) <= max(10 * err_o, 1e-9)


@pytest.mark.parametrize("n", [1, 2, 7])
def test_csr_degenerate_sizes(n, ctx):
    """A 1 x 1 system, a pair, and a path of 7 rows (tridiagonal)."""
    a = np.zeros((n, n))
    for i in range(n):
        a[i, i] = 2.5 + 0.1 * i
        if i + 1 < n:
            a[i, i + 1] = a[i + 1, i] = -1.0
    Ah = oracle.csr_from_dense(a)
    colour, nc = W.greedy_colouring(Ah.rp, Ah.col)
    Ah = oracle.CSR(n, Ah.rp, Ah.col, Ah.val, colour, nc)
    A = gpu_matrix(Ah)
    rng = np.random.default_rng(n)
    x_true = rng.random(n) + 0.5
    b = a @ x_true
    x0 = x_true * (1.0 + 0.2 * rng.random(n))
    say("csr degenerate", n)
    assert np.array_equal(host(lcs.residual(A, dev(b), dev(x0), ctx=ctx)), oracle.residual(Ah, b, x0))
    xd = np.linalg.solve(a, b)
    for pc in ("jacobi", "rbsgs"):
        for call in ("global", "residual", "gradient"):
            x = dev(x0)
            o = lcs.Options(eps=1e-10, precond=pc)
            if call == "global":
                lcs.solve_global(A, dev(b), x, o, ctx=ctx)
            else:
                lcs.solve_local_then_global(A, dev(b), x, call, "relmax", 0.3, 1, o, ctx=ctx)
            xg = host(x)
            assert np.linalg.norm(oracle.residual(Ah, b, xg)) <= 1.0001e-10 * np.linalg.norm(b)
            assert np.linalg.norm(xg - xd) / np.linalg.norm(xd) <= 1e-9


def _bad(kind):
    """Malformed CSR structures; every row pointer and column stays inside
    the arrays handed over, so the check reads nothing out of bounds."""
    Ah, _ = irregular(9, 7, 5)
    rp, col, val = Ah.rp.copy(), Ah.col.copy(), Ah.val.copy()
    colour, nc = Ah.colour.copy(), Ah.ncolours
    n = Ah.n
    if kind == "unsorted":
        col[rp[3]], col[rp[3] + 1] = col[rp[3] + 1], col[rp[3]]
    elif kind == "no_diag":
        k = int(np.nonzero(col[rp[4]:rp[5]] == 4)[0][0]) + rp[4]
        col, val = np.delete(col, k), np.delete(val, k)
        rp[5:] -= 1
    elif kind == "col_range":
        col[rp[6]] = n + 5
    elif kind == "ends":
        col, val = np.append(col, 0), np.append(val, 1.0)
    elif kind == "ptr_order":
        rp[10], rp[11] = rp[11], rp[10]
    elif kind == "empty_row":
        k0, k1 = rp[8], rp[9]
        col, val = np.delete(col, np.arange(k0, k1)), np.delete(val, np.arange(k0, k1))
        rp[9:] -= k1 - k0
    elif kind == "colour_clash":
        colour[col[rp[2]]] = colour[2] if col[rp[2]] != 2 else colour[col[rp[2] + 1]]
    elif kind == "colour_range":
        colour[0] = nc
    elif kind == "nan_value":
        val[rp[3] + 1] = np.nan
    elif kind == "inf_value":
        val[rp[7]] = -np.inf
    elif kind == "zero_diag":
        val[rp[4] + int(np.nonzero(col[rp[4]:rp[5]] == 4)[0][0])] = 0.0
    elif kind == "neg_diag":
        val[rp[6] + int(np.nonzero(col[rp[6]:rp[7]] == 6)[0][0])] = -2.0
    elif kind == "long_row":
        m = 80
        a = np.eye(m) * 100.0
        a[0, 1:70] = a[1:70, 0] = -1.0     # row 0: 70 entries
        B = oracle.csr_from_dense(a)
        rp, col, val = B.rp, B.col, B.val
        colour, nc = W.greedy_colouring(rp, col)
    return lcs.CsrMatrix(dev(rp, torch.int32), dev(col, torch.int32), dev(val),
                         dev(colour.astype(np.uint8), torch.uint8), nc)


@pytest.mark.parametrize("kind", ["unsorted", "no_diag", "col_range", "ends", "ptr_order",
                                  "empty_row", "colour_clash", "colour_range", "long_row",
                                  "nan_value", "inf_value", "zero_diag", "neg_diag"])
def test_csr_malformed_structure_rejected(kind, ctx):
    """Malformed structures and values are refused by the check before any
    work: LCS_EINVAL, or LCS_ENONFINITE for a NaN / infinite value; x is
    unchanged."""
    A = _bad(kind)
    say("csr malformed", kind)
    b = dev(np.ones(A.n))
    x0 = np.full(A.n, 0.25)
    x = dev(x0)
    with pytest.raises(lcs.LcsError) as e:
        lcs.solve_local_then_global(A, b, x, "residual", "relmax", 1e-3, 1, lcs.Options(eps=1e-10),
                                    ctx=ctx)
    want = lcs.ENONFINITE if kind in ("nan_value", "inf_value") else lcs.EINVAL
    assert e.value.status == want
    assert "CSR matrix" in str(e.value)
    assert np.array_equal(host(x), x0)


def test_csr_zero_diagonal_of_nonsymmetric_input_rejected(ctx):
    """Non-symmetric input accepts a negative diagonal but not a zero one
    (the Jacobi scaling divides by it)."""
    Ah, _ = irregular(9, 7, 5)
    val = Ah.val.copy()
    k4 = Ah.rp[4] + int(np.nonzero(Ah.col[Ah.rp[4]:Ah.rp[5]] == 4)[0][0])
    for v, ok in ((0.0, False), (-50.0, True)):
        val[k4] = v
        A = lcs.CsrMatrix(dev(Ah.rp, torch.int32), dev(Ah.col, torch.int32), dev(val), nonsym=True)
        y = dev(np.zeros(A.n))
        if ok:
            lcs.spmv(A, dev(np.ones(A.n)), y, ctx=ctx)
        else:
            with pytest.raises(lcs.LcsError) as e:
                lcs.spmv(A, dev(np.ones(A.n)), y, ctx=ctx)
            assert e.value.status == lcs.EINVAL and "zero diagonal" in str(e.value)


def test_csr_option_errors_and_context_reuse(ctx):
    """RB-SGS and GS sweeps need a colouring; after the errors the same
    context solves a valid system."""
    Ah, A, b, x0 = make_case("irr8")
    plain = gpu_matrix(oracle.CSR(Ah.n, Ah.rp, Ah.col, Ah.val, None, 0), coloured=False)
    say("csr option errors")
    x = dev(x0)
    with pytest.raises(lcs.LcsError) as e:
        lcs.solve_global(plain, dev(b), x, lcs.Options(precond="rbsgs"), ctx=ctx)
    assert e.value.status == lcs.EINVAL
    with pytest.raises(lcs.LcsError) as e:
        lcs.gs_sweeps(plain, dev(b), x, 1, ctx=ctx)
    assert e.value.status == lcs.EINVAL
    with pytest.raises(lcs.LcsError) as e:
        lcs.solve_global(_bad("unsorted"), dev(np.ones(63)), dev(np.zeros(63)), ctx=ctx)
    assert e.value.status == lcs.EINVAL
    assert np.array_equal(host(x), x0)
    lcs.solve_local_then_global(A, dev(b), x, "residual", "relmax", 1e-3, 1, lcs.Options(eps=1e-10),
                                ctx=ctx)
    assert np.linalg.norm(oracle.residual(Ah, b, host(x))) <= 1.0001e-10 * np.linalg.norm(b)


def test_csr_reuse_of_the_checked_copy(ctx):
    """reuse = True on the matrix the context copied last gives the copying
    call's result bit for bit; on another matrix (other addresses) the call
    checks and copies it, so it is solved correctly; a malformed matrix is
    still rejected."""
    Ah, A, b, x0 = make_case("irr16")
    Bh, B, bb, y0 = make_case("grid7")
    say("csr reuse")

    def run(M, rhs, z0):
        x = dev(z0)
        st = lcs.solve_local_then_global(M, dev(rhs), x, "residual", "relmax", 1e-3, 1,
                                         lcs.Options(eps=1e-10, precond="rbsgs"), ctx=ctx)
        return host(x), (st.K, st.its_local, st.its_global)

    ref, sref = run(A, b, x0)
    A.reuse = True
    for _ in range(2):
        got, sgot = run(A, b, x0)
        assert np.array_equal(got, ref) and sgot == sref
    B.reuse = True                      # not the context's copy: checked and copied
    yb, _ = run(B, bb, y0)
    assert np.linalg.norm(oracle.residual(Bh, bb, yb)) <= 1.0001e-10 * np.linalg.norm(bb)
    got, sgot = run(A, b, x0)           # A again: B's copy replaced it, so A is copied again
    assert np.array_equal(got, ref) and sgot == sref
    bad = _bad("unsorted")
    bad.reuse = True
    with pytest.raises(lcs.LcsError) as e:
        lcs.solve_global(bad, dev(np.ones(bad.n)), dev(np.zeros(bad.n)), ctx=ctx)
    assert e.value.status == lcs.EINVAL


def test_csr_streaming_operator_large(ctx):
    """A five-point matrix of 1600 x 1600 given in CSR: its FP64 pass exceeds
    the last-level cache, so the ELL copy is read with non-temporal loads.
    Per-row kernels bit-exact; Algorithm 1 meets the criterion."""
    nx = ny = 1600
    coef = W.assemble_5pt(W.lognormal_logk((ny, nx), 1.0, 21), 0.25)
    Ah = oracle.csr_from_stencil(W.KIND_5PT, nx, ny, 1, coef)
    A = gpu_matrix(Ah)
    yy, xx = np.mgrid[0:ny, 0:nx]
    x_true = (0.2 + 0.1 * np.sin(xx / 70.0) * np.cos(yy / 50.0)).ravel()
    b = oracle.spmv(Ah, x_true)
    x0 = x_true.copy()
    x0[((xx - 500) ** 2 + (yy - 800) ** 2 < 40 ** 2).ravel()] += 0.5
    say("csr streaming", A.n)
    assert np.array_equal(host(lcs.residual(A, dev(b), dev(x0), ctx=ctx)), oracle.residual(Ah, b, x0))
    assert np.array_equal(host(lcs.gradient(A, dev(x0), ctx=ctx)), oracle.gradient(Ah, x0))
    y = torch.empty(A.n, dtype=torch.float64, device=DEV)
    lcs.spmv(A, dev(x0), y, ctx=ctx)
    assert np.array_equal(host(y), oracle.spmv(Ah, x0))
    d = oracle.build_local_domain(Ah, b, x0, oracle.MODE_RESIDUAL, 1e-3, oracle.TH_RELMAX, 1)
    x = dev(x0)
    st = lcs.solve_local_then_global(A, dev(b), x, "residual", "relmax", 1e-3, 1,
                                     lcs.Options(eps=1e-10), ctx=ctx)
    assert st.K == d.K
    assert np.linalg.norm(oracle.residual(Ah, b, host(x))) <= 1.0001e-10 * np.linalg.norm(b)
    # the FP32 instantiation of the streaming operator (mixed precision) and
    # the colour-ordered SGS preconditioner on it: the domain equals the
    # oracle's, the criterion holds as the oracle recomputes it, and the
    # results agree with the FP64 Jacobi solve to within the criterion's reach
    x64 = host(x)
    nb = np.linalg.norm(b)
    for precond in ("jacobi", "rbsgs"):
        x = dev(x0)
        st = lcs.solve_local_then_global(A, dev(b), x, "residual", "relmax", 1e-3, 1,
                                         lcs.Options(eps=1e-10, precision="mixed", precond=precond),
                                         ctx=ctx)
        xg = host(x)
        rel = np.linalg.norm(oracle.residual(Ah, b, xg)) / nb
        dif = np.linalg.norm(xg - x64) / np.linalg.norm(x64)
        say(f"  mixed {precond}: K={st.K} its={st.its_local}+{st.its_global} relres={rel:.1e} "
            f"vs fp64 {dif:.1e}")
        assert st.K == d.K
        assert rel <= 1.0001e-10
        assert dif <= 1e-9


# ---- non-symmetric CSR input: GMRES(m) ----
def nonsym_case(nx=57, ny=43, seed=31, coloured=True):
    rp, col, val = W.irregular_nonsym(nx, ny, seed)
    colour, nc = W.greedy_colouring(rp, col)
    Ah = oracle.CSR(nx * ny, rp, col, val, colour if coloured else None, nc if coloured else 0)
    A = gpu_matrix(Ah, coloured)
    A.nonsym = True
    yy, xx = np.mgrid[0:ny, 0:nx]
    x_true = (0.2 + 0.1 * np.sin(xx / 7.0) * np.cos(yy / 5.0)).ravel()
    b = oracle.spmv(Ah, x_true)
    x0 = x_true.copy()
    x0[((xx - nx / 3) ** 2 + (yy - ny / 2) ** 2 < (min(nx, ny) / 6) ** 2).ravel()] += 0.5
    return Ah, A, b, x0


def gm(**kw):
    return oracle.Options(krylov=oracle.KRYLOV_GMRES, **kw)


@pytest.mark.parametrize("coloured", [True, False])
@pytest.mark.parametrize("mode,thresh,theta", [("residual", "relmax", 1e-3),
                                               ("residual", "paper", 1e-10),
                                               ("gradient", "relmax", 1e-3)])
def test_csr_nonsym_local_then_global_gmres(coloured, mode, thresh, theta, ctx):
    Ah, A, b, x0 = nonsym_case(coloured=coloured)
    say("csr nonsym local_then_global", coloured, mode, thresh)
    om = {"residual": oracle.MODE_RESIDUAL, "gradient": oracle.MODE_GRADIENT}[mode]
    ot = {"relmax": oracle.TH_RELMAX, "paper": oracle.TH_PAPER}[thresh]
    xo, so, _ = oracle.local_then_global(Ah, b, x0, om, theta, ot, 1, gm(eps=1e-10))
    x = dev(x0)
    st = lcs.solve_local_then_global(A, dev(b), x, mode, thresh, theta, 1, lcs.Options(eps=1e-10),
                                     ctx=ctx)
    xg = host(x)
    nb = np.linalg.norm(b)
    assert abs(st.K - so.K) <= (2 if thresh == "paper" else 0)
    assert abs(st.its_local - so.its_local) <= 2
    assert np.linalg.norm(oracle.residual(Ah, b, xg)) <= 1.0001e-10 * nb
    xd = np.linalg.solve(Ah.dense(), b)
    err_g = np.linalg.norm(xg - xd) / np.linalg.norm(xd)
    err_o = np.linalg.norm(xo - xd) / np.linalg.norm(xd)
    say(f"  K={st.K} its {st.its_local}+{st.its_global} (oracle {so.its_local}+{so.its_global}) "
        f"err {err_g:.1e} / {err_o:.1e}")
    assert err_g <= max(10 * err_o, 1e-10)


@pytest.mark.parametrize("pc", ["jacobi", "none"])
def test_csr_nonsym_gmres_trajectory(pc, ctx):
    """GMRES(4) stopped after k steps (k = 11 crosses two restarts): global
    solve against the oracle's GMRES; Algorithm 1 with k steps in the local
    and the global solve against the oracle's Algorithm 1."""
    Ah, A, b, x0 = nonsym_case()
    opc = {"jacobi": oracle.PC_JACOBI, "none": oracle.PC_NONE}[pc]
    for k in (3, 11):
        say("csr nonsym trajectory", pc, k)
        o = lcs.Options(eps=1e-30, precond=pc, max_iter=k, restart=4, max_outer=0)
        x = dev(x0)
        with pytest.raises(lcs.LcsError) as e:
            lcs.solve_global(A, dev(b), x, o, ctx=ctx)
        assert e.value.status == lcs.ENOCONV
        xk, _, itk, _ = oracle.gmres(Ah, b, x0, opc, m=4, tol_abs=0.0, max_iter=k)
        assert itk == k
        assert np.linalg.norm(host(x) - xk) / np.linalg.norm(xk) <= 1e-10
        x = dev(x0)
        with pytest.raises(lcs.LcsError) as e:
            lcs.solve_local_then_global(A, dev(b), x, "residual", "relmax", 1e-3, 1, o, ctx=ctx)
        assert e.value.status == lcs.ENOCONV
        xo, _, _ = oracle.local_then_global(Ah, b, x0, oracle.MODE_RESIDUAL, 1e-3, oracle.TH_RELMAX, 1,
                                            gm(eps=1e-30, max_iter=k, gmres_m=4, pc=opc))
        assert np.linalg.norm(host(x) - xo) / np.linalg.norm(xo) <= 1e-10


def test_csr_nonsym_option_errors(ctx):
    Ah, A, b, x0 = nonsym_case()
    say("csr nonsym option errors")
    x = dev(x0)
    for o in [lcs.Options(precision="mixed"), lcs.Options(precond="rbsgs"), lcs.Options(restart=0)]:
        with pytest.raises(lcs.LcsError) as e:
            lcs.solve_global(A, dev(b), x, o, ctx=ctx)
        assert e.value.status == lcs.EINVAL
    assert np.array_equal(host(x), x0)


def test_csr_nonsym_streaming_large(ctx):
    """The non-symmetric nine-point operator of 1600 x 1600 given in CSR: its
    pass exceeds the last-level cache, so GMRES runs on the streaming ELL
    operator.  Per-row kernels bit-exact; Algorithm 1 and the global GMRES
    meet the criterion."""
    nx = ny = 1600
    coef = W.assemble_9n(nx, ny, 0.25, speed=2.0)
    Ah = oracle.csr_from_stencil(W.KIND_9N, nx, ny, 1, coef)
    A = gpu_matrix(Ah)
    A.nonsym = True
    yy, xx = np.mgrid[0:ny, 0:nx]
    x_true = (0.2 + 0.1 * np.sin(xx / 70.0) * np.cos(yy / 50.0)).ravel()
    b = oracle.spmv(Ah, x_true)
    x0 = x_true.copy()
    x0[((xx - 500) ** 2 + (yy - 800) ** 2 < 40 ** 2).ravel()] += 0.5
    say("csr nonsym streaming", A.n)
    assert np.array_equal(host(lcs.residual(A, dev(b), dev(x0), ctx=ctx)), oracle.residual(Ah, b, x0))
    nb = np.linalg.norm(b)
    for call in ("local", "global"):
        x = dev(x0)
        if call == "local":
            lcs.solve_local_then_global(A, dev(b), x, "residual", "paper", 1e-10, 1,
                                        lcs.Options(eps=1e-10), ctx=ctx)
        else:
            lcs.solve_global(A, dev(b), x, lcs.Options(eps=1e-10), ctx=ctx)
        assert np.linalg.norm(oracle.residual(Ah, b, host(x))) <= 1.0001e-10 * nb, call
