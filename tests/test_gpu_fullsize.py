"""Full-size parity: the configurations' own sizes, in the launch configuration
the benchmark times.

Every input comes from the generators and the oracle: the oracle evolves the
sequences (64^2, 1024^2), or, at 16.8M unknowns, makes the previous state x_0
with one global solve of system 0 that both sides then start system 1 from.
Checked:
  * the local domain bit for bit (max-norm-relative threshold), or within the
    near-tie band of the paper threshold (its ||b|| is summed in another order),
  * the returned x meets ||b - A x|| <= 1e-10 ||b|| recomputed by the oracle in
    FP64 at full size,
  * the solution's error against a tight reference x* (the oracle's PCG to
    1e-14 ||b||, continued from the oracle's own Algorithm 1 solution), next
    to the oracle's own error: the GPU's at most 10x the oracle's, or 1e-10
    (FP64) / 1e-9 (FP32 inner solves with FP64 refinement).  At 16.8M
    unknowns the oracle runs in its OpenMP build (bit-identical to the
    serial one), and the mixed-precision result is also checked against the
    GPU's FP64 solve within kappa * 2 eps.
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


def say(*a):
    print("[case]", *a, flush=True)


def dev(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype).to(DEV)


def host(t):
    return t.detach().cpu().numpy()


def kappa_bound(Ah, dt):
    """kappa(A) <= lambda_max / lambda_min with lambda_max <= max_i sum_j |a_ij|
    (Gershgorin) and lambda_min >= 1/dt (A = I/dt + a positive semidefinite
    diffusion part)."""
    absA = oracle.CSR(Ah.n, Ah.rp, Ah.col, np.abs(Ah.val))
    return float(np.max(oracle.spmv(absA, np.ones(Ah.n)))) * dt


def check_domain(A_gpu, Ah, b, x0, thresh, theta, e_max, ctx, mode="residual"):
    idx, mask, st = lcs.build_local_domain(A_gpu, dev(b), dev(x0), mode, thresh, theta, e_max,
                                           want_mask=True, ctx=ctx)
    om = oracle.MODE_RESIDUAL if mode == "residual" else oracle.MODE_GRADIENT
    ot = {"relmax": oracle.TH_RELMAX, "paper": oracle.TH_PAPER}[thresh]
    d = oracle.build_local_domain(Ah, b, x0, om, theta, ot, e_max)
    if thresh == "relmax":
        assert st.K == d.K and st.tau == d.tau and st.e_rounds == d.rounds
        assert np.array_equal(host(idx), d.idx)
        assert np.array_equal(host(mask), d.mask)
    else:
        band = Ah.n * np.finfo(np.float64).eps * d.tau
        assert abs(st.tau - d.tau) <= band
        diff = np.nonzero(host(mask) != d.mask)[0]
        assert len(diff) <= 4
        for i in diff:
            assert abs(abs(d.score[i]) - d.tau) <= 2 * band
    return d


def test_c1_picard_64x64():
    """64x64 five-point Picard sequence, REL_MAX theta = 1e-3, E_max = 1."""
    w = W.c1_picard()
    say("c1", w.name)
    Ah = oracle.csr_from_stencil(w.kind, w.nx, w.ny, w.nz, w.coef)
    A = lcs.matrix_from_numpy(w.kind, w.nx, w.ny, w.nz, w.coef, DEV)
    ctx = lcs.Context()
    x_prev = w.x_start.copy()
    for s in range(w.n_systems):
        b = w.rhs(s, x_prev)
        if np.linalg.norm(b - oracle.spmv(Ah, x_prev)) == 0.0:
            break
        check_domain(A, Ah, b, x_prev, "relmax", 1e-3, 1, ctx)
        x = dev(x_prev)
        st = lcs.solve_local_then_global(A, dev(b), x, "residual", "relmax", 1e-3, 1, ctx=ctx)
        xg = host(x)
        nb = np.linalg.norm(b)
        assert np.linalg.norm(oracle.residual(Ah, b, xg)) <= 1.0001e-10 * nb
        xo, so, _ = oracle.local_then_global(Ah, b, x_prev, oracle.MODE_RESIDUAL, 1e-3,
                                             oracle.TH_RELMAX, 1, oracle.Options(eps=1e-10))
        assert st.K == so.K and abs(st.its_local - so.its_local) <= 1
        xd = oracle.pcg(Ah, b, xo, oracle.PC_JACOBI, 1e-14 * nb, 5000)[0]
        e_g = np.linalg.norm(xg - xd) / np.linalg.norm(xd)
        e_o = np.linalg.norm(xo - xd) / np.linalg.norm(xd)
        say(f"  picard {s}: K={st.K} its={st.its_local}+{st.its_global} err={e_g:.1e} (oracle {e_o:.1e})")
        assert e_g <= max(10 * e_o, 1e-10)
        x_prev = xo          # the oracle carries the sequence


def _oracle_sequence(Ah, dt, src, n_steps, pc=oracle.PC_JACOBI):
    """x_{k-1}, b_k of the first systems, evolved by the oracle."""
    xs, bs = [np.zeros(Ah.n)], []
    for k in range(n_steps):
        b = xs[-1] * (1.0 / dt) + src(k)
        x, st = oracle.solve_global(Ah, b, xs[-1], oracle.Options(eps=1e-10, pc=pc))
        assert st.status == oracle.OK
        bs.append(b)
        xs.append(x)
    return xs, bs


def test_c2_1024_full():
    """1024^2 five-point FP64, the benchmark's configuration: systems 1..3."""
    w = W.c2_moving_disk()
    say("c2", w.name)
    Ah = oracle.csr_from_stencil(w.kind, w.nx, w.ny, w.nz, w.coef)
    A = lcs.matrix_from_numpy(w.kind, w.nx, w.ny, w.nz, w.coef, DEV)
    ctx = lcs.Context()
    opts = lcs.Options(eps=1e-10)
    src = lambda k: W.disk_source(w.nx, w.ny, w.nx / 4.0 + 4.0 * k, w.ny / 2.0, 40.0, 1.0)
    xs, bs = _oracle_sequence(Ah, w.dt, src, 4)
    for k in range(1, 4):
        b, x0 = bs[k], xs[k]
        check_domain(A, Ah, b, x0, "relmax", 1e-3, 1, ctx)
        check_domain(A, Ah, b, x0, "paper", 1e-10, 1, ctx)
        check_domain(A, Ah, b, x0, "relmax", 1e-4, 0, ctx, mode="gradient")
        x = dev(x0)
        st = lcs.solve_local_then_global(A, dev(b), x, "residual", "paper", 1e-10, 1, opts, ctx=ctx)
        xg = host(x)
        nb = np.linalg.norm(b)
        assert np.linalg.norm(oracle.residual(Ah, b, xg)) <= 1.0001e-10 * nb
        xo, so, _ = oracle.local_then_global(Ah, b, x0, oracle.MODE_RESIDUAL, 1e-10,
                                             oracle.TH_PAPER, 1, oracle.Options(eps=1e-10))
        xd = oracle.pcg(Ah, b, xo, oracle.PC_JACOBI, 1e-14 * nb, 5000)[0]
        e_g = np.linalg.norm(xg - xd) / np.linalg.norm(xd)
        e_o = np.linalg.norm(xo - xd) / np.linalg.norm(xd)
        say(f"  system {k}: K={st.K} (oracle {so.K}) its={st.its_local}+{st.its_global} "
            f"err={e_g:.1e} (oracle {e_o:.1e})")
        assert abs(st.K - so.K) <= 4
        assert e_g <= max(10 * e_o, 1e-10)


def _big_case(w, src, opts, pc_oracle):
    """System 1 of a 16.8M sequence, from the oracle's solution of system 0:
    domain parity at full size, the FP64 criterion by the oracle, and the
    error of the GPU's Algorithm 1 (mixed and FP64 inner solves) against the
    oracle's tight reference, next to the oracle's own Algorithm 1."""
    A = lcs.matrix_from_numpy(w.kind, w.nx, w.ny, w.nz, w.coef, DEV,
                              with32=opts.precision == "mixed")
    ctx = lcs.Context()
    theta = 0.1 * opts.eps       # the benchmark's threshold: 0.1 eps ||b|| / sqrt(N)
    oracle.set_parallel(True)
    try:
        say(f"  oracle CSR and state x_0 ({oracle.threads()} threads)")
        Ah = oracle.csr_from_stencil(w.kind, w.nx, w.ny, w.nz, w.coef)
        b0 = src(0)
        x0, st0 = oracle.solve_global(Ah, b0, np.zeros(Ah.n), oracle.Options(eps=1e-8, pc=pc_oracle))
        assert st0.status == oracle.OK
        b = x0 * (1.0 / w.dt) + src(1)
        nb = np.linalg.norm(b)
        say("  domains")
        check_domain(A, Ah, b, x0, "relmax", 1e-3, 1, ctx)
        check_domain(A, Ah, b, x0, "paper", 1e-10, 1, ctx)
        check_domain(A, Ah, b, x0, "paper", theta, 1, ctx)
        say("  oracle Algorithm 1 and tight reference")
        pc = oracle.PC_SGS if opts.precond == "rbsgs" else oracle.PC_JACOBI
        xo, so, _ = oracle.local_then_global(Ah, b, x0, oracle.MODE_RESIDUAL, theta, oracle.TH_PAPER,
                                             1, oracle.Options(eps=1e-10, pc=pc))
        xd = oracle.pcg(Ah, b, xo, pc, 1e-14 * nb, 5000)[0]
        e_o = np.linalg.norm(xo - xd) / np.linalg.norm(xd)
        results = {}
        for prec in (opts.precision, "fp64"):
            o = lcs.Options(**{**opts.__dict__, "precision": prec})
            x = dev(x0)
            st = lcs.solve_local_then_global(A, dev(b), x, "residual", "paper", theta, 1, o, ctx=ctx)
            xg = host(x)
            rel = np.linalg.norm(oracle.residual(Ah, b, xg)) / nb
            e_g = np.linalg.norm(xg - xd) / np.linalg.norm(xd)
            say(f"  {prec}: K={st.K} (oracle {so.K}) its={st.its_local}+{st.its_global} "
                f"outer={st.n_outer} relres={rel:.2e} err vs x*={e_g:.2e} (oracle's own {e_o:.2e})")
            assert rel <= 1.0001e-10
            assert abs(st.K - so.K) <= 4
            assert e_g <= max(10 * e_o, 1e-9 if prec == "mixed" else 1e-10)
            results[prec] = xg
    finally:
        oracle.set_parallel(False)
    # property: the mixed-precision result and the GPU's FP64 global solve to
    # 1e-12 (both meeting the criterion) agree within kappa * 2 eps
    x64 = dev(x0)
    lcs.solve_global(A, dev(b), x64, lcs.Options(eps=1e-12, precond=opts.precond), ctx=ctx)
    err = np.linalg.norm(results[opts.precision] - host(x64)) / np.linalg.norm(host(x64))
    bound = max(1e-9, kappa_bound(Ah, w.dt) * 2e-10)
    say(f"  mixed local-then-global vs FP64 global (1e-12): {err:.2e} (bound {bound:.1e})")
    assert err <= bound


@pytest.mark.timeout(600)
def test_c3_4096_mixed_full():
    """4096^2 nine-point anisotropic, FP32 inner + FP64 refinement."""
    w = W.c3_aniso_front(n_systems=2)
    say("c3", w.name)
    src = lambda k: W.disk_source(w.nx, w.ny, w.nx / 4.0 + 8.0 * k, w.ny / 2.0, 350.0, 1.0)
    _big_case(w, src, lcs.Options(eps=1e-10, precision="mixed"), oracle.PC_JACOBI)


@pytest.mark.timeout(600)
def test_c5_256cube_mixed_rbsgs_full():
    """256^3 seven-point, sigma 1.5, FP32 inner RB-SGS + FP64 refinement."""
    w = W.c5_sphere3d(n_systems=2)
    say("c5", w.name)
    src = lambda k: W.ball_source(w.nx, w.ny, w.nz, w.nx / 4.0 + 2.0 * k, w.ny / 2.0, w.nz / 2.0,
                                  20.0, 1.0)
    _big_case(w, src, lcs.Options(eps=1e-10, precision="mixed", precond="rbsgs"), oracle.PC_JACOBI)
