"""Contexts on a caller-owned workspace (lcs_create_with_workspace): the
buffer comes from torch.empty(lcs_workspace_bytes(A, opts), dtype=uint8), and
every call gives the bit-identical result of a context that owns its
buffers, without allocating device memory; a workspace that is too small is
refused before any work."""
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


def ws_for(nbytes):
    return torch.empty(nbytes, dtype=torch.uint8, device=DEV)


def sequence_c2(n_sys=3):
    """The first systems of the 1024^2 five-point sequence: (A, [b_k], [x_(k-1)])."""
    w = W.c2_moving_disk()
    A = lcs.matrix_from_numpy(w.kind, w.nx, w.ny, w.nz, w.coef, DEV, with32=True)
    ctx = lcs.Context()
    x = torch.zeros(w.n, dtype=torch.float64, device=DEV)
    bs, xs = [], []
    for k in range(n_sys):
        b = x * (1.0 / w.dt) + dev(W.disk_source(w.nx, w.ny, w.nx / 4.0 + 4.0 * k, w.ny / 2.0,
                                                 40.0, 1.0))
        xs.append(x.clone())
        lcs.solve_global(A, b, x, lcs.Options(eps=1e-10), ctx=ctx)
        bs.append(b)
    ctx.close()
    return w, A, bs, xs


CALLS = [
    ("paper residual", lambda A, b, x, o, c: lcs.solve_local_then_global(
        A, b, x, "residual", "paper", 1e-10, 1, o, ctx=c)),
    ("relmax residual", lambda A, b, x, o, c: lcs.solve_local_then_global(
        A, b, x, "residual", "relmax", 1e-3, 1, o, ctx=c)),
    ("gradient", lambda A, b, x, o, c: lcs.solve_local_then_global(
        A, b, x, "gradient", "relmax", 1e-4, 0, o, ctx=c)),
    ("global", lambda A, b, x, o, c: lcs.solve_global(A, b, x, o, ctx=c)),
]


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_c2_systems_on_caller_workspace_match_owned_context(precision):
    """1024^2 systems: Algorithm 1 (three domain kinds) and the global PCG on
    a workspace context equal the owning context's results bit for bit, and
    no call changes the device's free memory."""
    w, A, bs, xs = sequence_c2()
    o = lcs.Options(eps=1e-10, precision=precision)
    nb = lcs.workspace_bytes(A, o)
    say(f"c2 {precision}: workspace {nb / 2**20:.1f} MiB")
    assert nb >= 60 * w.n, nb
    ws = ws_for(nb)
    own, wsc = lcs.Context(), lcs.Context(workspace=ws)
    x = torch.empty(w.n, dtype=torch.float64, device=DEV)
    y = torch.empty_like(x)
    # the owning context first (it grows its buffers as K grows), keeping results
    ref = {}
    for k in range(len(bs)):
        for name, call in CALLS:
            x.copy_(xs[k])
            ref[k, name] = (call(A, bs[k], x, o, own), x.clone())
    torch.cuda.synchronize()
    # then the workspace context alone, into preallocated result vectors (no
    # torch allocation in between): the device's free memory must not move
    got = {key: torch.empty_like(x) for key in ref}
    sts = {}
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    for k in range(len(bs)):
        for name, call in CALLS:
            y.copy_(xs[k])
            sts[k, name] = call(A, bs[k], y, o, wsc)
            got[k, name].copy_(y)
    torch.cuda.synchronize()
    free1 = torch.cuda.mem_get_info()[0]
    say(f"free device memory before {free0} after {free1}")
    assert free1 == free0
    for (k, name), (s1, x1) in ref.items():
        s2 = sts[k, name]
        say(f"  system {k} {name}: K={s2.K} its={s2.its_local}+{s2.its_global}")
        assert torch.equal(x1, got[k, name]), (k, name)
        assert (s1.K, s1.e_rounds, s1.its_local, s1.its_global, s1.n_outer) == \
               (s2.K, s2.e_rounds, s2.its_local, s2.its_global, s2.n_outer), (k, name)
        assert s2.relres_final <= 1e-10
    wsc.close()
    own.close()


def test_pieces_and_local_solve_on_workspace():
    """Domain construction, the restricted CSR, the local solve, residual,
    gradient and both SpMV precisions on a workspace context equal the owning
    context's results; the calls that need less accept a workspace sized for
    them alone."""
    dims = (131, 77, 1)
    nx, ny, _ = dims
    coef = W.assemble_9pt(nx, ny, 0.25, 100.0, 30.0)
    Ah = oracle.csr_from_stencil(W.KIND_9PT, nx, ny, 1, coef)
    rng = np.random.default_rng(3)
    xt = np.zeros(Ah.n)
    xt.reshape(ny, nx)[20:40, 30:70] = 1.0
    b = dev(oracle.spmv(Ah, xt))
    x0 = dev(xt * (1.0 + 0.3 * rng.random(Ah.n)))
    A = lcs.matrix_from_numpy(W.KIND_9PT, nx, ny, 1, coef, DEV)
    o = lcs.Options(eps=1e-10, precision="mixed")
    ws = ws_for(lcs.workspace_bytes(A, o))
    own, wsc = lcs.Context(), lcs.Context(workspace=ws)
    for mode, th, theta, e in [("residual", "relmax", 1e-3, 2), ("gradient", "relmax", 1e-2, 0)]:
        i1, m1, s1 = lcs.build_local_domain(A, b, x0, mode, th, theta, e, want_mask=True, ctx=own)
        i2, m2, s2 = lcs.build_local_domain(A, b, x0, mode, th, theta, e, want_mask=True, ctx=wsc)
        assert torch.equal(i1, i2) and torch.equal(m1, m2) and s1.tau == s2.tau
        r1, r2 = lcs.gather_restricted(A, i1, ctx=own), lcs.gather_restricted(A, i1, ctx=wsc)
        assert all(torch.equal(a, c) for a, c in zip(r1, r2))
        xa, xb = x0.clone(), x0.clone()
        lcs.solve_local(A, b, xa, i1, o, ctx=own)
        lcs.solve_local(A, b, xb, i1, o, ctx=wsc)
        assert torch.equal(xa, xb)
    assert torch.equal(lcs.residual(A, b, x0, ctx=own), lcs.residual(A, b, x0, ctx=wsc))
    assert torch.equal(lcs.gradient(A, x0, ctx=own), lcs.gradient(A, x0, ctx=wsc))
    y1, y2 = torch.empty_like(x0), torch.empty_like(x0)
    assert torch.equal(lcs.spmv(A, x0, y1, ctx=own), lcs.spmv(A, x0, y2, ctx=wsc))
    x32 = x0.float()
    z1, z2 = torch.empty_like(x32), torch.empty_like(x32)
    assert torch.equal(lcs.spmv(A, x32, z1, ctx=own), lcs.spmv(A, x32, z2, ctx=wsc))
    # a workspace of the fixed head alone serves the residual and SpMV
    small = lcs.Context(workspace=ws[: 1 << 20])
    assert torch.equal(lcs.residual(A, b, x0, ctx=small), lcs.residual(A, b, x0, ctx=own))
    small.close()
    wsc.close()
    own.close()


def test_too_small_workspace_is_refused_before_any_work():
    """One byte under lcs_workspace_bytes of the call: LCS_EINVAL naming the
    sizes, x unchanged; the context then serves a smaller problem."""
    nx, ny = 200, 150
    coef = W.assemble_5pt(W.lognormal_logk((ny, nx), 1.0, 5), 0.25)
    A = lcs.matrix_from_numpy(W.KIND_5PT, nx, ny, 1, coef, DEV)
    o = lcs.Options(eps=1e-10)
    need = lcs.workspace_bytes(A, o)
    ws = ws_for(need)
    tight = lcs.Context(workspace=ws[: need - 1])
    b = torch.ones(nx * ny, dtype=torch.float64, device=DEV)
    x = torch.zeros_like(b)
    with pytest.raises(lcs.LcsError) as e:
        lcs.solve_local_then_global(A, b, x, "residual", "paper", 1e-10, 1, o, ctx=tight)
    assert e.value.status == lcs.EINVAL and "workspace" in str(e.value)
    assert int(torch.count_nonzero(x)) == 0
    with pytest.raises(lcs.LcsError):
        lcs.solve_global(A, b, x, o, ctx=tight)
    assert int(torch.count_nonzero(x)) == 0
    # a smaller grid fits
    coef2 = W.assemble_5pt(W.lognormal_logk((100, 150), 1.0, 6), 0.25)
    A2 = lcs.matrix_from_numpy(W.KIND_5PT, 150, 100, 1, coef2, DEV)
    b2 = torch.ones(150 * 100, dtype=torch.float64, device=DEV)
    x2 = torch.zeros_like(b2)
    st = lcs.solve_local_then_global(A2, b2, x2, "residual", "paper", 1e-10, 1, o, ctx=tight)
    assert st.relres_final <= 1e-10
    tight.close()
    # misaligned and NULL workspaces
    with pytest.raises(lcs.LcsError):
        lcs.Context(workspace=ws[1:4097])
    with pytest.raises(lcs.LcsError):
        lcs.Context(workspace=ws[:64])


def test_csr_gmres_and_batched_on_workspace():
    """General sparse input (its ELL copy kept across calls with reuse, also
    after a stencil call on the same workspace), GMRES on the non-symmetric
    kind, and a batched call, each against an owning context."""
    rp, col, val = W.irregular_spd(60, 50, seed=11)
    colour, nc = W.greedy_colouring(rp, col)
    t = lambda a, dt: torch.as_tensor(np.ascontiguousarray(a)).to(dt).to(DEV)
    C = lcs.CsrMatrix(t(rp, torch.int32), t(col, torch.int32), t(val, torch.float64),
                      t(colour, torch.uint8), nc)
    n = C.n
    o = lcs.Options(eps=1e-10)
    ws = ws_for(lcs.workspace_bytes(C, o))
    own, wsc = lcs.Context(), lcs.Context(workspace=ws)
    rng = np.random.default_rng(5)
    b = dev(rng.random(n))
    x0 = dev(0.5 * rng.random(n))
    dims = (60, 50, 1)
    coefs = W.assemble_5pt(W.lognormal_logk((50, 60), 1.0, 8), 0.25)
    S = lcs.matrix_from_numpy(W.KIND_5PT, *dims, coefs, DEV)
    for rep in range(3):
        C.reuse = rep > 0
        xa, xb = x0.clone(), x0.clone()
        s1 = lcs.solve_local_then_global(C, b, xa, "residual", "relmax", 1e-2, 1, o, ctx=own)
        s2 = lcs.solve_local_then_global(C, b, xb, "residual", "relmax", 1e-2, 1, o, ctx=wsc)
        assert torch.equal(xa, xb) and s1.K == s2.K, rep
        # a stencil call in between uses the same workspace
        xs = x0.clone()
        lcs.solve_global(S, b, xs, o, ctx=wsc)
    wsc.close()
    # GMRES on the non-symmetric nine-point stencil
    nx, ny = 64, 48
    c9n = W.assemble_9n(nx, ny, 0.25, speed=2.0)
    A9 = lcs.matrix_from_numpy(W.KIND_9N, nx, ny, 1, c9n, DEV)
    og = lcs.Options(eps=1e-10, restart=20)
    wsg = lcs.Context(workspace=ws_for(lcs.workspace_bytes(A9, og)))
    bb = dev(rng.random(nx * ny))
    xa, xb = torch.zeros_like(bb), torch.zeros_like(bb)
    s1 = lcs.solve_local_then_global(A9, bb, xa, "residual", "paper", 1e-10, 1, og, ctx=own)
    s2 = lcs.solve_local_then_global(A9, bb, xb, "residual", "paper", 1e-10, 1, og, ctx=wsg)
    assert torch.equal(xa, xb) and (s1.its_local, s1.its_global) == (s2.its_local, s2.its_global)
    wsg.close()
    # batched: 5 systems of a five-point grid
    G = 5
    cb = torch.stack([dev(W.assemble_5pt(W.lognormal_logk((30, 40), 1.0, 20 + g), 0.25))
                      for g in range(G)])
    B = lcs.BatchMatrix(W.KIND_5PT, 40, 30, 1, cb)
    bg = dev(rng.random((G, 1200)))
    wsb = lcs.Context(workspace=ws_for(lcs.workspace_bytes_batched(B, G, o)))
    xa, xb = torch.zeros_like(bg), torch.zeros_like(bg)
    sa = lcs.solve_local_then_global_batched(B, bg, xa, "residual", "paper", 1e-10, 1, o, ctx=own)
    sb = lcs.solve_local_then_global_batched(B, bg, xb, "residual", "paper", 1e-10, 1, o, ctx=wsb)
    assert torch.equal(xa, xb) and [s.K for s in sa] == [s.K for s in sb]
    wsb.close()
    own.close()
