"""lcs_build_local_domain_static, the entry point for callers that cannot
allocate: called through the C ABI, its domain (idx, K, mask, tau, rounds)
equals lcs_build_local_domain's bit for bit, on two calls in a row (the
second on a smaller grid, so the shared scratch array holds the previous
call's larger contents), and it refuses what it cannot serve before any
work."""
import ctypes

import numpy as np
import pytest

from paper_2001_01158_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2001_01158_amd import lcs  # noqa: E402

DEV = "cuda:0"


def say(*a):
    print("[case]", *a, flush=True)


def system(kind, nx, ny, nz, seed):
    """A stencil system with a localized change: b = A x_true, x0 = x_true
    perturbed on a box."""
    if kind == W.KIND_5PT:
        coef = W.assemble_5pt(W.lognormal_logk((ny, nx), 1.0, seed), 0.25)
    elif kind == W.KIND_9PT:
        coef = W.assemble_9pt(nx, ny, 0.25, 100.0, 30.0)
    else:
        coef = W.assemble_7pt(W.lognormal_logk((nz, ny, nx), 1.0, seed), 0.25)
    A = lcs.matrix_from_numpy(kind, nx, ny, nz, coef, DEV)
    rng = np.random.default_rng(seed)
    n = nx * ny * nz
    xt = torch.as_tensor(rng.random(n) * 1e-3).to(DEV)
    g = xt.view(nz, ny, nx)
    g[:, ny // 3: ny // 3 + max(1, ny // 5), nx // 4: nx // 4 + max(1, nx // 5)] += 1.0
    b = torch.empty_like(xt)
    lcs.spmv(A, xt, b)
    x0 = xt.clone()
    x0.view(nz, ny, nx)[:, ny // 3: ny // 3 + max(1, ny // 5), nx // 4: nx // 4 + max(1, nx // 5)] *= 0.5
    return A, b, x0


def static_call(A, b, x0, mode, thresh, theta, e_max):
    """The C ABI call with caller-allocated outputs."""
    L = lcs.lib()
    idx = torch.full((A.n,), -7, dtype=torch.int32, device=DEV)
    mask = torch.full((A.n,), 0xAA, dtype=torch.uint8, device=DEV)
    K = ctypes.c_int64(-1)
    st = lcs._Stats()
    rc = L.lcs_build_local_domain_static(ctypes.byref(A.c()), ctypes.c_void_p(b.data_ptr()),
                                         ctypes.c_void_p(x0.data_ptr()), lcs._MODES[mode],
                                         lcs._THRESH[thresh], float(theta), int(e_max),
                                         ctypes.c_void_p(idx.data_ptr()),
                                         ctypes.c_void_p(mask.data_ptr()), ctypes.byref(K),
                                         ctypes.byref(st), lcs._stream())
    return rc, idx, mask, K.value, st


SETTINGS = [("residual", "relmax", 1e-3, 2), ("residual", "paper", 1e-10, 1),
            ("gradient", "relmax", 1e-2, 0)]


@pytest.mark.parametrize("kind, big, small", [
    (W.KIND_5PT, (2048, 1024, 1), (333, 201, 1)),          # the first at the 2^21-cell limit
    (W.KIND_9PT, (700, 650, 1), (97, 61, 1)),
    (W.KIND_7PT, (96, 80, 70), (23, 17, 11)),
])
def test_static_domain_matches_context_domain(kind, big, small):
    ctx = lcs.Context()
    for dims, seed in ((big, 1), (small, 2)):
        A, b, x0 = system(kind, *dims, seed)
        for mode, thresh, theta, e in SETTINGS:
            say(f"kind {kind} dims {dims} {mode} {thresh} {theta} e_max {e}")
            rc, idx, mask, K, st = static_call(A, b, x0, mode, thresh, theta, e)
            assert rc == lcs.OK, lcs.lib().lcs_last_error().decode()
            i_ref, m_ref, s_ref = lcs.build_local_domain(A, b, x0, mode, thresh, theta, e,
                                                         want_mask=True, ctx=ctx)
            assert K == i_ref.numel() == s_ref.K
            assert 0 < K < A.n
            assert torch.equal(idx[:K], i_ref)
            assert torch.equal(mask, m_ref)
            assert st.tau == s_ref.tau and st.e_rounds == s_ref.e_rounds and st.K == K
            assert int((idx[K:] != -7).sum()) == 0   # nothing written past K
    ctx.close()


def test_static_domain_refuses_what_it_cannot_serve():
    L = lcs.lib()
    # one cell over the limit: refused before any work, outputs untouched
    A, b, x0 = system(W.KIND_5PT, 2049, 1024, 1, 3)
    rc, idx, mask, K, _ = static_call(A, b, x0, "residual", "relmax", 1e-3, 1)
    assert rc == lcs.EINVAL and "2^21" in L.lcs_last_error().decode()
    assert K == -1 and int((idx != -7).sum()) == 0 and int((mask != 0xAA).sum()) == 0
    # general sparse input
    rp = torch.tensor([0, 1, 2], dtype=torch.int32, device=DEV)
    col = torch.tensor([0, 1], dtype=torch.int32, device=DEV)
    val = torch.tensor([2.0, 3.0], dtype=torch.float64, device=DEV)
    C = lcs.CsrMatrix(rp, col, val)
    rc, *_ = static_call(C, val.clone(), val.clone(), "residual", "relmax", 1e-3, 1)
    assert rc == lcs.EINVAL
    # bad arguments
    A, b, x0 = system(W.KIND_5PT, 64, 48, 1, 4)
    rc, *_ = static_call(A, b, x0, "residual", "relmax", -1.0, 1)
    assert rc == lcs.EINVAL
    rc, *_ = static_call(A, b, x0, "gradient", "paper", 1e-10, 1)
    assert rc == lcs.EINVAL
    # and a good call still works after the refusals
    rc, idx, mask, K, st = static_call(A, b, x0, "residual", "relmax", 1e-3, 1)
    i_ref, m_ref, _ = lcs.build_local_domain(A, b, x0, "residual", "relmax", 1e-3, 1, want_mask=True)
    assert rc == lcs.OK and K == i_ref.numel() and torch.equal(idx[:K], i_ref)
    assert torch.equal(mask, m_ref)
