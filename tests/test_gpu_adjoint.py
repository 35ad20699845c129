"""Adjoint of the local character-based solve vs the oracle's full-domain
FP64 adjoint and central finite differences."""
import numpy as np
import pytest

import oracle
from paper_2001_01158_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2001_01158_amd import lcs  # noqa: E402
from paper_2001_01158_amd.autograd import LocalSolve, SolveConfig  # noqa: E402

DEV = "cuda:0"


def say(*a):
    print("[case]", *a, flush=True)


def problem(kind, dims, seed, dt=4.0, window=None):
    nx, ny, nz = dims
    shape = (ny, nx) if kind == W.KIND_5PT else (nz, ny, nx)
    logk = W.lognormal_logk(shape, 1.0, seed)
    n = nx * ny * nz
    rng = np.random.default_rng(seed + 1)
    coef = (W.assemble_5pt if kind == W.KIND_5PT else W.assemble_7pt)(logk, 1.0 / dt)
    Ah = oracle.csr_from_stencil(kind, nx, ny, nz, coef)
    # previous state and a localized source: b = x_prev/dt + q
    x_prev = 0.1 + 0.01 * rng.random(n)
    q = np.zeros(n)
    q.reshape(nz, ny, nx)[nz // 3: nz // 3 + max(1, nz // 3), ny // 3: ny // 2, nx // 3: nx // 2] = 1.0
    b = x_prev / dt + q
    x_obs = oracle.pcg(Ah, b, x_prev, oracle.PC_JACOBI, 1e-13 * np.linalg.norm(b), 20000)[0] * 0.9
    win = np.zeros(n)
    if window is None:
        win.reshape(nz, ny, nx)[:, ny // 4: 3 * ny // 4, nx // 4: 3 * nx // 4] = 1.0
    else:
        win.reshape(nz, ny, nx)[window] = 1.0
    return logk, b, x_prev, x_obs, win, Ah


def oracle_adjoint(kind, dims, logk, b, x_prev, x_obs, win):
    """Full-domain FP64 adjoint: tight global solves for x and lambda."""
    nx, ny, nz = dims
    coef = oracle.assemble_logk(kind, nx, ny, nz, 0.25, logk)
    Ah = oracle.csr_from_stencil(kind, nx, ny, nz, coef)
    nb = np.linalg.norm(b)
    x = oracle.pcg(Ah, b, x_prev, oracle.PC_JACOBI, 1e-14 * nb, 50000)[0]
    g = win * (x - x_obs)
    lam = oracle.pcg(Ah, g, np.zeros_like(g), oracle.PC_JACOBI, 1e-14 * np.linalg.norm(g), 50000)[0]
    return x, lam, oracle.grad_logk(kind, nx, ny, nz, logk, x, lam)


def run_gpu(kind, dims, logk, b, x_prev, x_obs, win, eps, thresh="paper", theta=None):
    nx, ny, nz = dims
    cfg = SolveConfig(kind=kind, nx=nx, ny=ny, nz=nz, inv_dt=0.25, mode="residual", thresh=thresh,
                      theta=eps if theta is None else theta, e_max=1, opts=lcs.Options(eps=eps))
    lk = torch.tensor(logk, dtype=torch.float64, device=DEV, requires_grad=True)
    bb = torch.tensor(b, dtype=torch.float64, device=DEV, requires_grad=True)
    x = LocalSolve.apply(lk, bb, torch.tensor(x_prev, device=DEV), cfg, None)
    wv = torch.tensor(win, device=DEV)
    loss = 0.5 * torch.sum(wv * (x - torch.tensor(x_obs, device=DEV)) ** 2)
    loss.backward()
    return x.detach().cpu().numpy(), lk.grad.detach().cpu().numpy().reshape(-1), \
        bb.grad.detach().cpu().numpy(), cfg


@pytest.mark.parametrize("kind,dims", [(W.KIND_5PT, (64, 48, 1)), (W.KIND_7PT, (14, 12, 10))])
def test_adjoint_matches_full_domain_oracle(kind, dims):
    say("adjoint vs oracle", kind, dims)
    logk, b, x_prev, x_obs, win, Ah = problem(kind, dims, 31)
    xo, lamo, go = oracle_adjoint(kind, dims, logk, b, x_prev, x_obs, win)
    xg, gl, gb, _ = run_gpu(kind, dims, logk, b, x_prev, x_obs, win, eps=1e-13)
    assert np.linalg.norm(xg - xo) / np.linalg.norm(xo) < 1e-10
    assert np.linalg.norm(gb - lamo) / np.linalg.norm(lamo) < 1e-9
    assert np.linalg.norm(gl - go) / np.linalg.norm(go) < 1e-9


def test_adjoint_central_differences_small():
    kind, dims = W.KIND_5PT, (40, 32, 1)
    say("adjoint FD small")
    logk, b, x_prev, x_obs, win, Ah = problem(kind, dims, 41)
    xg, gl, gb, cfg = run_gpu(kind, dims, logk, b, x_prev, x_obs, win, eps=1e-14)

    def L(lk, bv):
        x = LocalSolve.apply(torch.tensor(lk, device=DEV), torch.tensor(bv, device=DEV),
                             torch.tensor(x_prev, device=DEV), cfg, None)
        return 0.5 * float(torch.sum(torch.tensor(win, device=DEV) *
                                     (x - torch.tensor(x_obs, device=DEV)) ** 2))

    rng = np.random.default_rng(5)
    h = 1e-6
    for _ in range(4):
        d = rng.choice([-1.0, 1.0], size=logk.shape)
        fd = (L(logk + h * d, b) - L(logk - h * d, b)) / (2 * h)
        ad = float(np.sum(gl * d.reshape(-1)))
        assert abs(fd - ad) <= 1e-6 * max(abs(ad), 1e-12) + 1e-9, (fd, ad)
        e = rng.choice([-1.0, 1.0], size=b.shape)
        fd = (L(logk, b + h * e) - L(logk, b - h * e)) / (2 * h)
        ad = float(np.sum(gb * e))
        assert abs(fd - ad) <= 1e-6 * max(abs(ad), 1e-12) + 1e-9, (fd, ad)


@pytest.mark.timeout(600)
def test_adjoint_c4_scale():
    """2048x2048 five-point FP64, loss over a 256x256 window: gradient of 4.2M
    log-conductivities and b, against the oracle's full-domain adjoint and
    central differences along 16 Rademacher directions.  The state and the
    observation come from oracle solves (system 2 of a C2-like sequence)."""
    nx = ny = 2048
    say("adjoint 2048^2")
    w = W.c4_adjoint(k_sys=2)
    logk = w.logk
    dims = (nx, ny, 1)
    Ah = oracle.csr_from_stencil(w.kind, nx, ny, 1, w.coef)
    x_prev = np.zeros(nx * ny)
    for k in range(2):
        q = W.disk_source(nx, ny, nx / 2.0 - 4.0 * 2 + 4.0 * k, ny / 2.0, 40.0, 1.0)
        x_prev, st = oracle.solve_global(Ah, x_prev * 0.25 + q, x_prev, oracle.Options(eps=1e-10))
        assert st.status == oracle.OK
    q = W.disk_source(nx, ny, nx / 2.0, ny / 2.0, 40.0, 1.0)
    b = x_prev * 0.25 + q
    win = np.zeros(nx * ny)
    c0 = nx // 2 - 128
    win.reshape(ny, nx)[c0:c0 + 256, c0:c0 + 256] = 1.0
    logk2 = W.lognormal_logk((ny, nx), 1.0, W.BASE_SEED + 4)
    A2h = oracle.csr_from_stencil(w.kind, nx, ny, 1, W.assemble_5pt(logk2, 0.25))
    x_obs, st = oracle.solve_global(A2h, b, x_prev, oracle.Options(eps=1e-12))
    assert st.status == oracle.OK
    say("  gpu forward/backward")
    xg, gl, gb, cfg = run_gpu(W.KIND_5PT, dims, logk, b, x_prev, x_obs, win, eps=1e-13)
    say("  oracle full-domain adjoint")
    xo, lamo, go = oracle_adjoint(W.KIND_5PT, dims, logk, b, x_prev, x_obs, win)
    ex = np.linalg.norm(xg - xo) / np.linalg.norm(xo)
    eb = np.linalg.norm(gb - lamo) / np.linalg.norm(lamo)
    el = np.linalg.norm(gl - go) / np.linalg.norm(go)
    say(f"  rel err x {ex:.2e}  dL/db {eb:.2e}  dL/dlogk {el:.2e}")
    assert ex < 1e-9 and eb < 1e-8 and el < 1e-8
    say("  central differences")

    def L(lk, bv):
        x = LocalSolve.apply(torch.tensor(lk, device=DEV), torch.tensor(bv, device=DEV),
                             torch.tensor(x_prev, device=DEV), cfg, None)
        return 0.5 * float(torch.sum(torch.tensor(win, device=DEV) *
                                     (x - torch.tensor(x_obs, device=DEV)) ** 2))

    rng = np.random.default_rng(16)
    h = 1e-6
    worst = 0.0
    for _ in range(16):
        d = rng.choice([-1.0, 1.0], size=logk.shape)
        fd = (L(logk + h * d, b) - L(logk - h * d, b)) / (2 * h)
        ad = float(np.sum(gl * d.reshape(-1)))
        worst = max(worst, abs(fd - ad) / max(abs(ad), 1e-30))
    say(f"  worst FD relative gap over 16 directions: {worst:.2e}")
    assert worst < 1e-4


def _adjoint_256(logk, x_prev, b, centre, seed):
    """The 256^3 adjoint checks at one step: loss over a 32^3 window around
    `centre`, forward and adjoint at eps = 1e-13 (FP32 inner RB-SGS + FP64
    refinement); properties recomputed by the oracle at full size and
    central differences along 4 Rademacher directions."""
    n1, kind, dt = 256, W.KIND_7PT, 4.0
    n = n1 ** 3
    cx, cy, cz = centre
    zz, yy, xx = np.meshgrid(*(np.arange(n1, dtype=np.float64),) * 3, indexing="ij")
    bump = np.exp(-((xx - cx) ** 2 + (yy - cy) ** 2 + (zz - cz) ** 2) / 200.0)
    x_obs = (x_prev.reshape(n1, n1, n1) + 0.5 * bump).reshape(-1)
    del zz, yy, xx, bump
    win = np.zeros(n)
    x0_, y0_, z0_ = (int(round(c)) - 16 for c in (cx, cy, cz))
    win.reshape(n1, n1, n1)[z0_:z0_ + 32, y0_:y0_ + 32, x0_:x0_ + 32] = 1.0
    eps = 1e-13
    opts = lcs.Options(eps=eps, precision="mixed", precond="rbsgs")
    cfg = SolveConfig(kind=kind, nx=n1, ny=n1, nz=n1, inv_dt=1.0 / dt, mode="residual",
                      thresh="paper", theta=eps, e_max=1, opts=opts)
    lk = torch.tensor(logk.reshape(-1), dtype=torch.float64, device=DEV, requires_grad=True)
    bb = torch.tensor(b, dtype=torch.float64, device=DEV, requires_grad=True)
    xp = torch.tensor(x_prev, device=DEV)
    wv, xo = torch.tensor(win, device=DEV), torch.tensor(x_obs, device=DEV)
    say("  gpu forward/backward")
    x = LocalSolve.apply(lk, bb, xp, cfg, None)
    loss = 0.5 * torch.sum(wv * (x - xo) ** 2)
    loss.backward()
    xg = host_np(x)
    gl, gb = host_np(lk.grad), host_np(bb.grad)
    say("  oracle checks")
    coef = oracle.assemble_logk(kind, n1, n1, n1, 1.0 / dt, logk)
    cg = host_np(lcs.assemble_logk(kind, n1, n1, n1, 1.0 / dt, lk.detach()))
    ca = coef.reshape(cg.shape)
    assert np.max(np.abs(cg - ca) / np.maximum(np.abs(ca), 1e-300)) <= 1e-14
    Ah = oracle.csr_from_stencil(kind, n1, n1, n1, ca)
    del cg, ca, coef
    # eps holds on the GPU's own operator; the oracle's differs by the
    # rounding of exp, so allow 1e-11 here
    assert np.linalg.norm(oracle.residual(Ah, b, xg)) <= 1e-11 * np.linalg.norm(b)
    g = win * (xg - x_obs)
    assert np.linalg.norm(oracle.residual(Ah, g, gb)) <= 1e-11 * np.linalg.norm(g)
    go = oracle.grad_logk(kind, n1, n1, n1, logk, xg, gb)
    el = np.linalg.norm(gl - go) / np.linalg.norm(go)
    say(f"  grad log k against the oracle's formula: {el:.2e}")
    assert el <= 1e-12
    del Ah, go
    say("  central differences")

    def L(lkv):
        xx_ = LocalSolve.apply(lkv, bb.detach(), xp, cfg, None)
        return 0.5 * float(torch.sum(wv * (xx_ - xo) ** 2))

    rng = np.random.default_rng(seed)
    h = 1e-6
    worst = 0.0
    base = lk.detach()
    for _ in range(4):
        d = torch.tensor(rng.choice([-1.0, 1.0], size=n), device=DEV)
        fd = (L(base + h * d) - L(base - h * d)) / (2 * h)
        ad = float(np.sum(gl * host_np(d)))
        worst = max(worst, abs(fd - ad) / max(abs(ad), 1e-30))
    say(f"  worst FD relative gap over 4 directions: {worst:.2e}")
    assert worst < 1e-4


@pytest.mark.timeout(600)
def test_adjoint_c5_scale():
    """256^3 seven-point, sigma = 1.5, FP32 inner RB-SGS + FP64 refinement:
    the adjoint of one step with the loss over a 32^3 window at the front.
    A full-domain oracle adjoint at this size takes minutes on one core, so
    the checks are properties recomputed by the oracle at full size:
    * the GPU's assembly from log k matches the oracle's;
    * the forward x and the adjoint lambda meet their criteria;
    * grad log k equals the oracle's formula applied to that x and lambda;
    * central differences agree along 4 Rademacher directions.
    The previous state is the constant 0.1, which A maps to 0.1 / dt exactly
    (zero-flux faces), so r^(0) is the ball source itself."""
    n1, dt = 256, 4.0
    n = n1 ** 3
    say("adjoint 256^3, constant previous state")
    logk = W.lognormal_logk((n1, n1, n1), 1.5, W.BASE_SEED + 4)
    x_prev = np.full(n, 0.1)
    q = W.ball_source(n1, n1, n1, n1 / 2.0, n1 / 2.0, n1 / 2.0, 20.0, 1.0)
    _adjoint_256(logk, x_prev, x_prev / dt + q, (n1 / 2.0,) * 3, 25)


@pytest.mark.timeout(900)
def test_adjoint_c5_final_step():
    """The 256^3 sequence as the benchmark defines it: 50 backward-Euler
    systems with the ball source moving 2 cells per system, each solved by
    Algorithm 1 (FP32 inner RB-SGS + FP64 refinement to 1e-10, threshold
    0.1 eps ||b|| / sqrt(N)); the adjoint of the final step (system 49, from
    x_48), loss over a 32^3 window on the front, with the same checks."""
    w = W.c5_sphere3d()
    n1, dt = w.nx, w.dt
    assert w.n_systems == 50
    say("adjoint 256^3, final step of the 50-system sequence")
    A = lcs.matrix_from_numpy(w.kind, n1, n1, n1, w.coef, DEV, with32=True)
    ctx = lcs.Context()
    opts = lcs.Options(eps=1e-10, precision="mixed", precond="rbsgs")
    x = torch.zeros(w.n, dtype=torch.float64, device=DEV)
    centre = lambda k: (n1 / 4.0 + 2.0 * k, n1 / 2.0, n1 / 2.0)
    for k in range(w.n_systems - 1):
        b = x / dt + torch.as_tensor(W.ball_source(n1, n1, n1, *centre(k), 20.0, 1.0)).to(DEV)
        st = lcs.solve_local_then_global(A, b, x, "residual", "paper", 1e-11, 1, opts, ctx=ctx)
        assert st.relres_final <= 1e-10
        if k % 10 == 0 or k == w.n_systems - 2:
            say(f"  system {k}: K={st.K} its={st.its_local}+{st.its_global}")
    ctx.close()
    del A
    x_prev = host_np(x)
    kf = w.n_systems - 1
    b = x_prev / dt + W.ball_source(n1, n1, n1, *centre(kf), 20.0, 1.0)
    _adjoint_256(w.logk, x_prev, b, centre(kf), 26)


def host_np(t):
    return t.detach().cpu().numpy().reshape(-1)
