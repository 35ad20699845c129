"""CPU oracle of the local character-based method (ctypes over oracle.c).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
CPU-baseline leg of the benchmark, never by the product path.  It shares no
code with the HIP library.  Everything runs serially in FP64.

Functions follow the paper (Ye, An, Xu, arXiv 2001.01158):
  build_local_domain  Algorithm 2 (gradient) / Algorithm 3 (residual)
  restricted          eq. (BEFC) block B = A[Omega, Omega]
  solve_local         steps 3-7 of Algorithm 1 (eq. loc-equ, eq. sol-assemble,
                      Gauss-Seidel smoothing)
  solve_global        PCG to eq. (rel-res-conv-criteria)
  local_then_global   Algorithm 1
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_LIB_OMP = os.path.join(_HERE, "liboracle_omp.so")
# ORACLE_SANITIZE=1: load a build with AddressSanitizer and
# UndefinedBehaviorSanitizer instead (host code; run under
# LD_PRELOAD=libasan.so, as tests/test_oracle_sanitized.py does)
_SANITIZE = os.environ.get("ORACLE_SANITIZE") == "1"
if _SANITIZE:
    _LIB = os.path.join(_HERE, "liboracle_san.so")
_SAN_FLAGS = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
              "-fno-omit-frame-pointer", "-g"]

MODE_RESIDUAL, MODE_GRADIENT = 0, 1
TH_RELMAX, TH_ABS, TH_PAPER = 0, 1, 2
PC_NONE, PC_JACOBI, PC_SGS = 0, 1, 2
KRYLOV_CG, KRYLOV_GMRES = 0, 1
OK, EINVAL, ENOMEM, ENOCONV, EBREAKDOWN = 0, 1, 3, 4, 5


def _compile(out: str, extra: list):
    tmp = out + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math",
                           "-fPIC", "-shared"] + extra + ["-o", tmp, _SRC, "-lm"])
    os.replace(tmp, out)


def _stale(lib_path: str) -> bool:
    return not os.path.exists(lib_path) or os.path.getmtime(lib_path) < os.path.getmtime(_SRC)


def build(force: bool = True) -> str:
    """Compile oracle.c (no FP contraction, no fast-math): the serial checker
    liboracle.so and the OpenMP build liboracle_omp.so of the same source
    (row loops on all host cores, bit-identical results; timing only)."""
    if force or _stale(_LIB):
        _compile(_LIB, _SAN_FLAGS if _SANITIZE else [])
    if force or _stale(_LIB_OMP):
        _compile(_LIB_OMP, ["-fopenmp"])
    return _LIB


_lib = None
_lib_omp = None
_parallel = False


def set_parallel(on: bool) -> None:
    """Route every oracle call to the OpenMP build (True) or the serial
    build (False, the default and the checker the tests use)."""
    global _parallel
    _parallel = bool(on)


def threads() -> int:
    """Host threads of the build in use (1 for the serial one)."""
    return int(lib().orc_threads())

P = ctypes.c_void_p
I64 = ctypes.c_int64
I32 = ctypes.c_int
D = ctypes.c_double


class _Opts(ctypes.Structure):
    _fields_ = [("eps", D), ("tol_local", D), ("max_iter", I32), ("pc", I32),
                ("n_smooth", I32), ("max_restart", I32), ("krylov", I32), ("gmres_m", I32)]


class _Stats(ctypes.Structure):
    _fields_ = [("K", I64), ("its_local", I32), ("its_global", I32), ("restarts", I32),
                ("status_local", I32), ("relres_after_local", D), ("relres_final", D)]


def lib():
    global _lib, _lib_omp
    if _parallel:
        if _lib_omp is None:
            if _stale(_LIB_OMP):
                build(force=True)
            _lib_omp = _declare(ctypes.CDLL(_LIB_OMP))
        return _lib_omp
    if _lib is None:
        if _stale(_LIB):
            build(force=True)
        _lib = _declare(ctypes.CDLL(_LIB))
    return _lib


def _declare(L):
    """ctypes signatures of the oracle's exports."""
    L.orc_stencil_nnz.restype = I64
    L.orc_stencil_nnz.argtypes = [I32, I32, I32, I32]
    L.orc_csr_from_stencil.argtypes = [I32, I32, I32, I32, P, P, P, P]
    L.orc_grid_colours.argtypes = [I32, I32, I32, I32, P]
    L.orc_residual.argtypes = [I64, P, P, P, P, P, P]
    L.orc_residual.restype = None
    L.orc_spmv.argtypes = [I64, P, P, P, P, P]
    L.orc_spmv.restype = None
    L.orc_dot.argtypes = [I64, P, P]
    L.orc_dot.restype = D
    L.orc_norm2.argtypes = [I64, P]
    L.orc_norm2.restype = D
    L.orc_gradient.argtypes = [I64, P, P, P, P]
    L.orc_gradient.restype = None
    L.orc_build_local_domain.argtypes = [I64, P, P, P, P, P, I32, I32, D, I32, P, P, P, P, P, P]
    L.orc_restricted_nnz.argtypes = [I64, P, P, P, I64, P]
    L.orc_restricted_nnz.restype = I64
    L.orc_restricted.argtypes = [P, P, P, P, I64, P, P, P, P]
    L.orc_restricted.restype = None
    L.orc_pcg.argtypes = [I64, P, P, P, P, P, I32, P, I32, D, I32, P, P]
    L.orc_gmres.argtypes = [I64, P, P, P, P, P, I32, I32, D, I32, P, P]
    L.orc_gs_sweeps.argtypes = [I64, P, P, P, P, P, P, I32, I32]
    L.orc_gs_sweeps.restype = None
    L.orc_solve_global.argtypes = [I64, P, P, P, P, P, P, I32, P, P]
    L.orc_solve_local.argtypes = [I64, P, P, P, P, P, P, I64, P, I32, P, P]
    L.orc_assemble_logk.argtypes = [I32, I32, I32, I32, D, P, P]
    L.orc_grad_logk.argtypes = [I32, I32, I32, I32, P, P, P, P]
    L.orc_heat_assemble.argtypes = [I32, I32, D, D, D, D, P, P, P, P]
    L.orc_threads.restype = I32
    L.orc_threads.argtypes = []
    return L


def _p(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


@dataclasses.dataclass
class CSR:
    n: int
    rp: np.ndarray      # int64[n+1]
    col: np.ndarray     # int32[nnz]
    val: np.ndarray     # float64[nnz]
    colour: Optional[np.ndarray] = None   # int8[n] grid colouring
    ncolours: int = 0

    def dense(self) -> np.ndarray:
        a = np.zeros((self.n, self.n))
        for i in range(self.n):
            for k in range(self.rp[i], self.rp[i + 1]):
                a[i, self.col[k]] = self.val[k]
        return a


def csr_from_stencil(kind: int, nx: int, ny: int, nz: int, coef: np.ndarray) -> CSR:
    L = lib()
    n = nx * ny * nz
    coef = _f64(coef)
    assert coef.size % n == 0
    nnz = L.orc_stencil_nnz(kind, nx, ny, nz)
    rp = np.empty(n + 1, np.int64)
    col = np.empty(nnz, np.int32)
    val = np.empty(nnz, np.float64)
    st = L.orc_csr_from_stencil(kind, nx, ny, nz, _p(coef), _p(rp), _p(col), _p(val))
    if st != OK:
        raise ValueError(f"orc_csr_from_stencil status {st}")
    colour = np.empty(n, np.int8)
    ncol = L.orc_grid_colours(kind, nx, ny, nz, _p(colour))
    return CSR(n, rp, col, val, colour, ncol)


def csr_from_dense(a: np.ndarray) -> CSR:
    """Pattern = non-zero entries of a (tests of the worked example)."""
    n = a.shape[0]
    rp = np.zeros(n + 1, np.int64)
    cols, vals = [], []
    for i in range(n):
        nz = np.nonzero(a[i])[0]
        cols.extend(nz.tolist())
        vals.extend(a[i, nz].tolist())
        rp[i + 1] = len(cols)
    return CSR(n, rp, np.array(cols, np.int32), np.array(vals, np.float64), np.zeros(n, np.int8), 1)


def residual(A: CSR, b, x) -> np.ndarray:
    b, x = _f64(b), _f64(x)
    r = np.empty(A.n)
    lib().orc_residual(A.n, _p(A.rp), _p(A.col), _p(A.val), _p(b), _p(x), _p(r))
    return r


def spmv(A: CSR, x) -> np.ndarray:
    x = _f64(x)
    y = np.empty(A.n)
    lib().orc_spmv(A.n, _p(A.rp), _p(A.col), _p(A.val), _p(x), _p(y))
    return y


def gradient(A: CSR, x) -> np.ndarray:
    x = _f64(x)
    g = np.empty(A.n)
    lib().orc_gradient(A.n, _p(A.rp), _p(A.col), _p(x), _p(g))
    return g


def norm2(v) -> float:
    v = _f64(v)
    return lib().orc_norm2(v.size, _p(v))


@dataclasses.dataclass
class Domain:
    idx: np.ndarray      # int32[K] ascending
    mask: np.ndarray     # uint8[n] round stamps (0 = outside)
    K: int
    rounds: int
    tau: float
    score: np.ndarray    # r^(0) or g


def build_local_domain(A: CSR, b, x0, mode: int = MODE_RESIDUAL, theta: float = 1e-3,
                       thresh: int = TH_RELMAX, e_max: int = 1) -> Domain:
    b, x0 = _f64(b), _f64(x0)
    n = A.n
    mask = np.zeros(n, np.uint8)
    idx = np.zeros(max(n, 1), np.int32)
    K = ctypes.c_int64(0)
    rounds = ctypes.c_int(0)
    tau = ctypes.c_double(0.0)
    score = np.zeros(n)
    st = lib().orc_build_local_domain(n, _p(A.rp), _p(A.col), _p(A.val), _p(b), _p(x0), mode,
                                      thresh, theta, e_max, _p(mask), _p(idx), ctypes.byref(K),
                                      ctypes.byref(rounds), ctypes.byref(tau), _p(score))
    if st != OK:
        raise ValueError(f"orc_build_local_domain status {st}")
    return Domain(idx[:K.value].copy(), mask, K.value, rounds.value, tau.value, score)


def restricted(A: CSR, idx) -> CSR:
    idx = np.ascontiguousarray(idx, np.int32)
    K = idx.size
    inv = np.empty(A.n, np.int32)
    L = lib()
    nnz = L.orc_restricted_nnz(A.n, _p(A.rp), _p(A.col), _p(idx), K, _p(inv))
    brp = np.empty(K + 1, np.int64)
    bcol = np.empty(max(nnz, 1), np.int32)
    bval = np.empty(max(nnz, 1), np.float64)
    L.orc_restricted(_p(A.rp), _p(A.col), _p(A.val), _p(idx), K, _p(inv), _p(brp), _p(bcol), _p(bval))
    colour = A.colour[idx].copy() if A.colour is not None else None
    return CSR(K, brp, bcol[:nnz].copy(), bval[:nnz].copy(), colour, A.ncolours)


def pcg(A: CSR, b, x0, pc: int = PC_JACOBI, tol_abs: float = 1e-10, max_iter: int = 10000):
    """Returns (x, status, iterations, recursive residual norm)."""
    b = _f64(b)
    x = _f64(x0).copy()
    it = ctypes.c_int(0)
    res = ctypes.c_double(0.0)
    colour = A.colour if A.colour is not None else np.zeros(A.n, np.int8)
    st = lib().orc_pcg(A.n, _p(A.rp), _p(A.col), _p(A.val), _p(b), _p(x), pc, _p(colour),
                       max(A.ncolours, 1), tol_abs, max_iter, ctypes.byref(it), ctypes.byref(res))
    return x, st, it.value, res.value


def gmres(A: CSR, b, x0, pc: int = PC_JACOBI, m: int = 40, tol_abs: float = 1e-10,
          max_iter: int = 10000):
    """Restarted GMRES(m), right-preconditioned.  Returns (x, status,
    iterations, last residual estimate)."""
    b = _f64(b)
    x = _f64(x0).copy()
    it = ctypes.c_int(0)
    res = ctypes.c_double(0.0)
    st = lib().orc_gmres(A.n, _p(A.rp), _p(A.col), _p(A.val), _p(b), _p(x), pc, m, tol_abs,
                         max_iter, ctypes.byref(it), ctypes.byref(res))
    return x, st, it.value, res.value


def gs_sweeps(A: CSR, b, x, n_sweeps: int = 1) -> np.ndarray:
    b = _f64(b)
    x = _f64(x).copy()
    lib().orc_gs_sweeps(A.n, _p(A.rp), _p(A.col), _p(A.val), _p(b), _p(x), _p(A.colour),
                        A.ncolours, n_sweeps)
    return x


@dataclasses.dataclass
class Options:
    eps: float = 1e-10
    tol_local: Optional[float] = None     # default: eps
    max_iter: int = 20000
    pc: int = PC_JACOBI
    n_smooth: int = 1
    max_restart: int = 3
    krylov: int = KRYLOV_CG       # KRYLOV_GMRES for a non-symmetric A
    gmres_m: int = 40             # GMRES restart length

    def c(self) -> _Opts:
        return _Opts(self.eps, self.eps if self.tol_local is None else self.tol_local,
                     self.max_iter, self.pc, self.n_smooth, self.max_restart, self.krylov,
                     self.gmres_m)


@dataclasses.dataclass
class Stats:
    status: int
    K: int = 0
    its_local: int = 0
    its_global: int = 0
    restarts: int = 0
    relres_after_local: float = float("nan")
    relres_final: float = float("nan")
    rounds: int = 0
    tau: float = 0.0


def _stats(st: int, s: _Stats) -> Stats:
    return Stats(st, s.K, s.its_local, s.its_global, s.restarts, s.relres_after_local, s.relres_final)


def solve_global(A: CSR, b, x0, opts: Options = Options()):
    b = _f64(b)
    x = _f64(x0).copy()
    s = _Stats()
    o = opts.c()
    st = lib().orc_solve_global(A.n, _p(A.rp), _p(A.col), _p(A.val), _p(b), _p(x), _p(A.colour),
                                A.ncolours, ctypes.byref(o), ctypes.byref(s))
    return x, _stats(st, s)


def solve_local(A: CSR, b, x0, idx, opts: Options = Options()):
    b = _f64(b)
    x = _f64(x0).copy()
    idx = np.ascontiguousarray(idx, np.int32)
    s = _Stats()
    o = opts.c()
    st = lib().orc_solve_local(A.n, _p(A.rp), _p(A.col), _p(A.val), _p(b), _p(x), _p(idx), idx.size,
                               _p(A.colour), A.ncolours, ctypes.byref(o), ctypes.byref(s))
    return x, _stats(st, s)


def local_then_global(A: CSR, b, x0, mode: int = MODE_RESIDUAL, theta: float = 1e-3,
                      thresh: int = TH_RELMAX, e_max: int = 1, opts: Options = Options()):
    """Algorithm 1: construct Omega, solve the local system, assemble, smooth,
    check eq. (rel-res-conv-criteria), else finish with the global solve.

    An x0 that already meets eq. (rel-res-conv-criteria) is the solution and
    comes back unchanged with K = 0 and an empty domain: the paper's
    algorithm presumes an x0 that is not yet converged, and the global solve
    (Krylov methods generally) stops at once on such an x0."""
    b = _f64(b)
    x0 = _f64(x0)
    r0n = float(np.linalg.norm(residual(A, b, x0)))
    bn = float(np.linalg.norm(b))
    if r0n <= opts.eps * bn:
        rel = r0n / bn if bn > 0 else r0n
        st = Stats(status=OK, relres_after_local=rel, relres_final=rel)
        dom = Domain(np.zeros(0, np.int32), np.zeros(A.n, np.uint8), 0, 0, 0.0, np.zeros(A.n))
        return x0.copy(), st, dom
    dom = build_local_domain(A, b, x0, mode, theta, thresh, e_max)
    x, sl = solve_local(A, b, x0, dom.idx, opts)
    if sl.relres_after_local <= opts.eps:
        sl.relres_final = sl.relres_after_local
        sl.rounds, sl.tau = dom.rounds, dom.tau
        return x, sl, dom
    x, sg = solve_global(A, b, x, opts)
    sg.K, sg.its_local, sg.relres_after_local = sl.K, sl.its_local, sl.relres_after_local
    sg.rounds, sg.tau = dom.rounds, dom.tau
    return x, sg, dom


def assemble_logk(kind: int, nx: int, ny: int, nz: int, inv_dt: float, logk) -> np.ndarray:
    logk = _f64(logk).reshape(-1)
    n = nx * ny * nz
    narr = 3 if kind == 0 else 4
    coef = np.empty(narr * n)
    st = lib().orc_assemble_logk(kind, nx, ny, nz, inv_dt, _p(logk), _p(coef))
    if st != OK:
        raise ValueError(f"orc_assemble_logk status {st}")
    return coef.reshape(narr, n)


def grad_logk(kind: int, nx: int, ny: int, nz: int, logk, x, lam) -> np.ndarray:
    logk, x, lam = _f64(logk).reshape(-1), _f64(x), _f64(lam)
    g = np.empty(nx * ny * nz)
    st = lib().orc_grad_logk(kind, nx, ny, nz, _p(logk), _p(x), _p(lam), _p(g))
    if st != OK:
        raise ValueError(f"orc_grad_logk status {st}")
    return g


def heat_assemble(nx: int, ny: int, inv_dt: float, power: float, tl: float, tr: float, tlin, told):
    """Picard system of the 2-D heat-conduction test (Section 3.1):
    (coef [3, N] of A with k = T_lin^power, b from T_old)."""
    tlin, told = _f64(tlin).reshape(-1), _f64(told).reshape(-1)
    n = nx * ny
    coef, b = np.empty(3 * n), np.empty(n)
    st = lib().orc_heat_assemble(nx, ny, inv_dt, power, tl, tr, _p(tlin), _p(told), _p(coef), _p(b))
    if st != OK:
        raise ValueError(f"orc_heat_assemble status {st}")
    return coef.reshape(3, n), b
