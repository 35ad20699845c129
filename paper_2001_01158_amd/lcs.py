"""Python binding of the C ABI in include/lcs.h (argument marshalling only).

Tensors are torch device tensors (FP64 vectors of length N, int32 index
arrays); the binding passes their data pointers and the current HIP stream to
liblcs.so.  Every step of the method runs in the library's kernels.  There is
no fallback: if the library is missing or fails to load, the import raises.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
from typing import Optional

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblcs.so")

OK, EINVAL, EHIP, ENOMEM, ENOCONV, EBREAKDOWN, ENONFINITE = range(7)
STENCIL5_2D, STENCIL9_2D, STENCIL7_3D, STENCIL9N_2D, CSR = 0, 1, 2, 3, 4
MODE_RESIDUAL, MODE_GRADIENT = 0, 1
THRESH_REL_MAX, THRESH_ABS, THRESH_PAPER = 0, 1, 2
PC_NONE, PC_JACOBI, PC_RBSGS = 0, 1, 2
PREC_FP64, PREC_MIXED = 0, 1
N_ARRAYS = {STENCIL5_2D: 3, STENCIL9_2D: 5, STENCIL7_3D: 4, STENCIL9N_2D: 9}

_MODES = {"residual": MODE_RESIDUAL, "gradient": MODE_GRADIENT}
_THRESH = {"relmax": THRESH_REL_MAX, "abs": THRESH_ABS, "paper": THRESH_PAPER}
_PC = {"none": PC_NONE, "jacobi": PC_JACOBI, "rbsgs": PC_RBSGS}
_PREC = {"fp64": PREC_FP64, "mixed": PREC_MIXED}

EXPORTED = ["lcs_default_options", "lcs_create", "lcs_destroy", "lcs_last_error",
            "lcs_solve_global", "lcs_build_local_domain", "lcs_solve_local",
            "lcs_solve_local_then_global", "lcs_residual", "lcs_gradient", "lcs_spmv",
            "lcs_gather_restricted", "lcs_gs_sweeps", "lcs_cast_coef", "lcs_assemble_logk",
            "lcs_grad_logk", "lcs_set_kernel_timing", "lcs_get_kernel_timing",
            "lcs_set_tiling", "lcs_assemble_heat", "lcs_norm2_diff",
            "lcs_solve_global_batched", "lcs_solve_local_then_global_batched",
            "lcs_workspace_bytes", "lcs_workspace_bytes_batched", "lcs_create_with_workspace",
            "lcs_build_local_domain_static", "lcs_set_colour_blocking",
            "lcs_set_short_columns"]
(TIME_NONE, TIME_LOCAL_AP, TIME_LOCAL_UPDATE, TIME_GLOBAL_AP, TIME_GLOBAL_UPDATE, TIME_SMOOTH,
 TIME_SCORE) = range(7)


class LcsError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"lcs status {status}: {msg}")
        self.status = status


class _Matrix(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
                ("nz", ctypes.c_int32), ("coef", ctypes.c_void_p), ("coef32", ctypes.c_void_p),
                ("row_ptr", ctypes.c_void_p), ("col", ctypes.c_void_p), ("val", ctypes.c_void_p),
                ("nnz", ctypes.c_int64), ("colour", ctypes.c_void_p), ("n_colours", ctypes.c_int32),
                ("csr_reuse", ctypes.c_int32), ("csr_nonsym", ctypes.c_int32)]


class _Options(ctypes.Structure):
    _fields_ = [("eps", ctypes.c_double), ("tol_local", ctypes.c_double),
                ("inner_tol", ctypes.c_double), ("max_iter", ctypes.c_int32),
                ("precond", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("n_smooth", ctypes.c_int32), ("check_every", ctypes.c_int32),
                ("max_outer", ctypes.c_int32), ("restart", ctypes.c_int32)]


class _Stats(ctypes.Structure):
    _fields_ = [("K", ctypes.c_int64), ("e_rounds", ctypes.c_int32), ("its_local", ctypes.c_int32),
                ("its_global", ctypes.c_int32), ("n_outer", ctypes.c_int32), ("tau", ctypes.c_double),
                ("relres_after_local", ctypes.c_double), ("relres_final", ctypes.c_double),
                ("ms_construct", ctypes.c_double), ("ms_local", ctypes.c_double),
                ("ms_smooth", ctypes.c_double), ("ms_global", ctypes.c_double)]


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load liblcs.so and declare the ABI.  Raises if it is missing."""
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with `python -m paper_2001_01158_amd.build`")
    L = ctypes.CDLL(path)
    P, I32, I64, D = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    PM, PO, PS = ctypes.POINTER(_Matrix), ctypes.POINTER(_Options), ctypes.POINTER(_Stats)
    sig = {
        "lcs_default_options": (None, [PO]),
        "lcs_create": (I32, [ctypes.POINTER(P)]),
        "lcs_destroy": (None, [P]),
        "lcs_last_error": (ctypes.c_char_p, []),
        "lcs_solve_global": (I32, [P, PM, P, P, PO, PS, P]),
        "lcs_build_local_domain": (I32, [P, PM, P, P, I32, I32, D, I32, P, P,
                                         ctypes.POINTER(I64), PS, P]),
        "lcs_solve_local": (I32, [P, PM, P, P, P, I64, PO, PS, P]),
        "lcs_solve_local_then_global": (I32, [P, PM, P, P, I32, I32, D, I32, PO, PS, P]),
        "lcs_solve_global_batched": (I32, [P, PM, I32, P, P, PO, P, P]),
        "lcs_solve_local_then_global_batched": (I32, [P, PM, I32, P, P, I32, I32, D, I32, PO, P,
                                                      P]),
        "lcs_residual": (I32, [P, PM, P, P, P, P]),
        "lcs_gradient": (I32, [P, PM, P, P, P]),
        "lcs_spmv": (I32, [P, PM, P, P, I32, I32, P]),
        "lcs_gather_restricted": (I32, [P, PM, P, I64, P, P, P, ctypes.POINTER(I64), P]),
        "lcs_gs_sweeps": (I32, [P, PM, P, P, I32, P]),
        "lcs_cast_coef": (I32, [P, PM, P, P]),
        "lcs_assemble_logk": (I32, [P, I32, I32, I32, I32, D, P, P, P]),
        "lcs_grad_logk": (I32, [P, I32, I32, I32, I32, P, P, P, P, P]),
        "lcs_set_kernel_timing": (I32, [P, I32]),
        "lcs_get_kernel_timing": (I32, [P, ctypes.POINTER(D), ctypes.POINTER(I64)]),
        "lcs_set_tiling": (I32, [P, I32, I32]),
        "lcs_set_colour_blocking": (I32, [P, I32]),
        "lcs_set_short_columns": (I32, [P, I32]),
        "lcs_assemble_heat": (I32, [P, I32, I32, D, D, D, D, P, P, P, P, P]),
        "lcs_norm2_diff": (I32, [P, P, P, I64, ctypes.POINTER(D), P]),
        "lcs_workspace_bytes": (ctypes.c_size_t, [PM, PO]),
        "lcs_workspace_bytes_batched": (ctypes.c_size_t, [PM, I32, PO]),
        "lcs_create_with_workspace": (I32, [ctypes.POINTER(P), P, ctypes.c_size_t]),
        "lcs_build_local_domain_static": (I32, [PM, P, P, I32, I32, D, I32, P, P,
                                                ctypes.POINTER(I64), PS, P]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    return L


_lib: Optional[ctypes.CDLL] = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        _lib = load_library()
    return _lib


def _check(status: int):
    if status != OK:
        raise LcsError(status, lib().lcs_last_error().decode())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t: Optional[torch.Tensor]):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("expected a device tensor")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    return ctypes.c_void_p(t.data_ptr())


def _vec(t: torch.Tensor, n: int, dtype=torch.float64, name: str = "vector"):
    if t.dtype != dtype or t.numel() != n:
        raise ValueError(f"{name}: expected {dtype} with {n} elements, got {t.dtype} {t.numel()}")
    return _ptr(t)


# ---------------------------------------------------------------------------
@dataclasses.dataclass
class Matrix:
    """Symmetric structured-grid stencil (see include/lcs.h for the layout)."""
    kind: int
    nx: int
    ny: int
    nz: int
    coef: torch.Tensor                    # (n_arrays, N) float64, device
    coef32: Optional[torch.Tensor] = None  # (n_arrays, N) float32, device

    max_row = 9   # entries per row, at most

    @property
    def n(self) -> int:
        return self.nx * self.ny * self.nz

    @property
    def device(self) -> torch.device:
        return self.coef.device

    def c(self) -> _Matrix:
        if self.coef.dtype != torch.float64 or self.coef.numel() != N_ARRAYS[self.kind] * self.n:
            raise ValueError("coef must be float64 of shape (n_arrays, N)")
        if self.coef32 is not None and (self.coef32.dtype != torch.float32
                                        or self.coef32.numel() != self.coef.numel()):
            raise ValueError("coef32 must be float32 of the same shape as coef")
        return _Matrix(self.kind, self.nx, self.ny, self.nz, _ptr(self.coef), _ptr(self.coef32))


@dataclasses.dataclass
class CsrMatrix:
    """General symmetric sparse matrix in CSR (columns strictly ascending in
    each row, diagonal stored, 1..64 entries per row), optionally with a
    colouring for the Gauss-Seidel sweeps; see include/lcs.h."""
    row_ptr: torch.Tensor                  # int32 [N + 1], device
    col: torch.Tensor                      # int32 [nnz], device
    val: torch.Tensor                      # float64 [nnz], device
    colour: Optional[torch.Tensor] = None  # uint8 [N], device
    n_colours: int = 0
    reuse: bool = False   # the arrays stay unchanged between calls: the context may
                          # keep its checked copy (sent only while the tensors' data
                          # pointers and versions are those of this context's last call)
    nonsym: bool = False  # not symmetric: solves use GMRES(m)
    kind = CSR
    max_row = 64
    _seen: dict = dataclasses.field(default_factory=dict, repr=False, compare=False)

    def _signature(self):
        ts = [self.row_ptr, self.col, self.val] + ([self.colour] if self.colour is not None else [])
        return tuple((t.data_ptr(), t._version) for t in ts)

    @property
    def n(self) -> int:
        return self.row_ptr.numel() - 1

    @property
    def device(self) -> torch.device:
        return self.val.device

    def c(self, ctx_key=None) -> _Matrix:
        """The C description.  ctx_key: the context the call goes to; csr_reuse
        is set only if reuse is on and no array was replaced or modified in
        place (torch's version counter) since this context's previous call."""
        if self.row_ptr.dtype != torch.int32 or self.col.dtype != torch.int32:
            raise ValueError("row_ptr and col must be int32")
        if self.val.dtype != torch.float64 or self.val.numel() != self.col.numel():
            raise ValueError("val must be float64 with one value per column index")
        if not (self.row_ptr.is_contiguous() and self.col.is_contiguous() and self.val.is_contiguous()):
            raise ValueError("row_ptr, col and val must be contiguous")
        if self.colour is not None and (self.colour.dtype != torch.uint8
                                        or self.colour.numel() != self.n
                                        or not self.colour.is_contiguous()):
            raise ValueError("colour must be contiguous uint8 of length N")
        m = _Matrix(CSR, self.n, 1, 1, None, None)
        m.row_ptr, m.col, m.val = _ptr(self.row_ptr), _ptr(self.col), _ptr(self.val)
        m.nnz = self.col.numel()
        m.colour, m.n_colours = _ptr(self.colour), int(self.n_colours)
        sig = self._signature()
        keep = self.reuse and ctx_key is not None and self._seen.get(ctx_key) == sig
        if ctx_key is not None:
            self._seen[ctx_key] = sig
        m.csr_reuse = 1 if keep else 0
        m.csr_nonsym = 1 if self.nonsym else 0
        return m


@dataclasses.dataclass
class Options:
    eps: float = 1e-10
    tol_local: float = 0.0
    inner_tol: float = 1e-5
    max_iter: int = 20000
    precond: str = "jacobi"
    precision: str = "fp64"
    n_smooth: int = 1
    check_every: int = 8
    max_outer: int = 10
    restart: int = 40        # GMRES(m) restart length (non-symmetric operator)

    def c(self) -> _Options:
        return _Options(self.eps, self.tol_local, self.inner_tol, self.max_iter, _PC[self.precond],
                        _PREC[self.precision], self.n_smooth, self.check_every, self.max_outer,
                        self.restart)


@dataclasses.dataclass
class Stats:
    K: int = 0
    e_rounds: int = 0
    its_local: int = 0
    its_global: int = 0
    n_outer: int = 0
    tau: float = 0.0
    relres_after_local: float = float("nan")
    relres_final: float = float("nan")
    ms_construct: float = 0.0
    ms_local: float = 0.0
    ms_smooth: float = 0.0
    ms_global: float = 0.0

    @staticmethod
    def of(s: _Stats) -> "Stats":
        return Stats(**{f: getattr(s, f) for f, _ in _Stats._fields_})


class Context:
    """A solver context (lcs_create / lcs_destroy).  Without `workspace` it
    owns grow-only device buffers.  With `workspace`, a caller-owned device
    tensor (for example torch.empty(workspace_bytes(A, opts), dtype=torch.uint8,
    device=...)), every device buffer of every call comes from that tensor
    (lcs_create_with_workspace) and no call allocates device memory; the
    context keeps a reference to the tensor until it is closed."""

    def __init__(self, workspace: Optional[torch.Tensor] = None):
        self._h = ctypes.c_void_p()
        self._ws = None
        if workspace is None:
            _check(lib().lcs_create(ctypes.byref(self._h)))
        else:
            if not workspace.is_contiguous():
                raise ValueError("workspace must be contiguous")
            nbytes = workspace.numel() * workspace.element_size()
            _check(lib().lcs_create_with_workspace(ctypes.byref(self._h), _ptr(workspace), nbytes))
            self._ws = workspace

    @property
    def handle(self):
        return self._h

    def close(self):
        if self._h:
            lib().lcs_destroy(self._h)
            self._h = ctypes.c_void_p()
        self._ws = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


_default_ctx: Optional[Context] = None


def default_context() -> Context:
    global _default_ctx
    if _default_ctx is None:
        _default_ctx = Context()
    return _default_ctx


def _ctx(ctx):
    return (ctx or default_context()).handle


def _mat(A, ctx):
    """A's C description for a call on ctx (general sparse input tracks, per
    context, whether its arrays changed since the previous call)."""
    if isinstance(A, CsrMatrix):
        return A.c(_ctx(ctx).value)
    return A.c()


def workspace_bytes(A, opts: Options = None) -> int:
    """Bytes of a caller-owned workspace serving every single-system call on
    A with opts (lcs_workspace_bytes; host arithmetic only)."""
    o = opts.c() if opts is not None else None
    nb = lib().lcs_workspace_bytes(ctypes.byref(A.c()), ctypes.byref(o) if o is not None else None)
    if nb == 0:
        raise LcsError(EINVAL, lib().lcs_last_error().decode())
    return int(nb)


def workspace_bytes_batched(A, G: int, opts: Options = None) -> int:
    """lcs_workspace_bytes_batched: the same for batched calls on G systems."""
    o = opts.c() if opts is not None else None
    nb = lib().lcs_workspace_bytes_batched(ctypes.byref(A.c()), int(G),
                                           ctypes.byref(o) if o is not None else None)
    if nb == 0:
        raise LcsError(EINVAL, lib().lcs_last_error().decode())
    return int(nb)


# ---------------------------------------------------------------------------
# the four calls of the method
# ---------------------------------------------------------------------------
def solve_global(A: Matrix, b: torch.Tensor, x: torch.Tensor, opts: Options = None,
                 ctx: Context = None) -> Stats:
    """Global PCG from x (in place) to ||b - A x|| <= eps ||b||."""
    opts = opts or Options()
    st = _Stats()
    o = opts.c()
    _check(lib().lcs_solve_global(_ctx(ctx), ctypes.byref(_mat(A, ctx)), _vec(b, A.n, name="b"),
                                  _vec(x, A.n, name="x"), ctypes.byref(o), ctypes.byref(st), _stream()))
    return Stats.of(st)


def build_local_domain(A: Matrix, b: torch.Tensor, x0: torch.Tensor, mode: str = "residual",
                       thresh: str = "relmax", theta: float = 1e-3, e_max: int = 1,
                       want_mask: bool = False, ctx: Context = None):
    """Algorithm 2 / 3.  Returns (idx[K] int32 device tensor, mask or None, Stats)."""
    idx = torch.empty(max(A.n, 1), dtype=torch.int32, device=b.device)
    mask = torch.empty(A.n, dtype=torch.uint8, device=b.device) if want_mask else None
    K = ctypes.c_int64(0)
    st = _Stats()
    _check(lib().lcs_build_local_domain(_ctx(ctx), ctypes.byref(_mat(A, ctx)), _vec(b, A.n, name="b"),
                                        _vec(x0, A.n, name="x0"), _MODES[mode], _THRESH[thresh],
                                        float(theta), int(e_max), _ptr(idx), _ptr(mask),
                                        ctypes.byref(K), ctypes.byref(st), _stream()))
    return idx[:K.value], mask, Stats.of(st)


STATIC_MAX_N = 1 << 21   # cells of lcs_build_local_domain_static


def build_local_domain_static(A: Matrix, b: torch.Tensor, x0: torch.Tensor, idx: torch.Tensor,
                              mode: str = "residual", thresh: str = "relmax", theta: float = 1e-3,
                              e_max: int = 1, mask: Optional[torch.Tensor] = None):
    """lcs_build_local_domain_static: Algorithm 2 / 3 with no context and no
    allocation; the caller passes idx (int32, capacity N) and optionally mask
    (uint8, N).  Returns (K, Stats)."""
    K = ctypes.c_int64(0)
    st = _Stats()
    if idx.dtype != torch.int32 or idx.numel() < A.n:
        raise ValueError("idx must be int32 with capacity N")
    if mask is not None and (mask.dtype != torch.uint8 or mask.numel() != A.n):
        raise ValueError("mask must be uint8 of length N")
    _check(lib().lcs_build_local_domain_static(ctypes.byref(A.c()), _vec(b, A.n, name="b"),
                                               _vec(x0, A.n, name="x0"), _MODES[mode],
                                               _THRESH[thresh], float(theta), int(e_max),
                                               _ptr(idx), _ptr(mask), ctypes.byref(K),
                                               ctypes.byref(st), _stream()))
    return K.value, Stats.of(st)


def solve_local(A: Matrix, b: torch.Tensor, x: torch.Tensor, idx: torch.Tensor,
                opts: Options = None, ctx: Context = None) -> Stats:
    """Steps 3-7 of Algorithm 1 on the given domain; x: in x^(0), out x~."""
    opts = opts or Options()
    if idx.dtype != torch.int32:
        raise ValueError("idx must be int32")
    idx = idx.contiguous()
    st = _Stats()
    o = opts.c()
    _check(lib().lcs_solve_local(_ctx(ctx), ctypes.byref(_mat(A, ctx)), _vec(b, A.n, name="b"),
                                 _vec(x, A.n, name="x"), _ptr(idx) if idx.numel() else None,
                                 idx.numel(), ctypes.byref(o), ctypes.byref(st), _stream()))
    return Stats.of(st)


def solve_local_then_global(A: Matrix, b: torch.Tensor, x: torch.Tensor, mode: str = "residual",
                            thresh: str = "relmax", theta: float = 1e-3, e_max: int = 1,
                            opts: Options = None, ctx: Context = None) -> Stats:
    """Algorithm 1; x: in x^(0), out the solution."""
    opts = opts or Options()
    st = _Stats()
    o = opts.c()
    _check(lib().lcs_solve_local_then_global(_ctx(ctx), ctypes.byref(_mat(A, ctx)), _vec(b, A.n, name="b"),
                                             _vec(x, A.n, name="x"), _MODES[mode], _THRESH[thresh],
                                             float(theta), int(e_max), ctypes.byref(o),
                                             ctypes.byref(st), _stream()))
    return Stats.of(st)


# ---------------------------------------------------------------------------
# batched solves: G systems on one grid (one workgroup each)
# ---------------------------------------------------------------------------
@dataclasses.dataclass
class BatchMatrix:
    """G stencil operators of one grid and kind: coef (G, n_arrays, N) float64."""
    kind: int
    nx: int
    ny: int
    nz: int
    coef: torch.Tensor

    @property
    def n(self) -> int:
        return self.nx * self.ny * self.nz

    @property
    def G(self) -> int:
        return self.coef.shape[0]

    def c(self) -> _Matrix:
        if (self.coef.dtype != torch.float64 or self.coef.dim() != 3
                or tuple(self.coef.shape[1:]) != (N_ARRAYS[self.kind], self.n)):
            raise ValueError("coef must be float64 of shape (G, n_arrays, N)")
        return _Matrix(self.kind, self.nx, self.ny, self.nz, _ptr(self.coef), None)


def _batch_stats(arr, G):
    return [Stats.of(arr[g]) for g in range(G)]


def solve_global_batched(A: BatchMatrix, b: torch.Tensor, x: torch.Tensor, opts: Options = None,
                         ctx: Context = None):
    """Global PCG of each of the G systems (b, x: (G, N)); x in place.
    Returns G Stats."""
    opts = opts or Options()
    G = A.G
    arr = (_Stats * G)()
    o = opts.c()
    _check(lib().lcs_solve_global_batched(_ctx(ctx), ctypes.byref(_mat(A, ctx)), G,
                                          _vec(b, G * A.n, name="b"), _vec(x, G * A.n, name="x"),
                                          ctypes.byref(o), arr, _stream()))
    return _batch_stats(arr, G)


def solve_local_then_global_batched(A: BatchMatrix, b: torch.Tensor, x: torch.Tensor,
                                    mode: str = "residual", thresh: str = "relmax",
                                    theta: float = 1e-3, e_max: int = 1, opts: Options = None,
                                    ctx: Context = None):
    """Algorithm 1 on each of the G systems (b, x: (G, N)); x in place.
    Returns G Stats."""
    opts = opts or Options()
    G = A.G
    arr = (_Stats * G)()
    o = opts.c()
    _check(lib().lcs_solve_local_then_global_batched(_ctx(ctx), ctypes.byref(_mat(A, ctx)), G,
                                                     _vec(b, G * A.n, name="b"),
                                                     _vec(x, G * A.n, name="x"), _MODES[mode],
                                                     _THRESH[thresh], float(theta), int(e_max),
                                                     ctypes.byref(o), arr, _stream()))
    return _batch_stats(arr, G)


# ---------------------------------------------------------------------------
# pieces of the path
# ---------------------------------------------------------------------------
def residual(A: Matrix, b: torch.Tensor, x: torch.Tensor, ctx: Context = None) -> torch.Tensor:
    r = torch.empty_like(b)
    _check(lib().lcs_residual(_ctx(ctx), ctypes.byref(_mat(A, ctx)), _vec(b, A.n, name="b"),
                              _vec(x, A.n, name="x"), _ptr(r), _stream()))
    return r


def gradient(A: Matrix, x: torch.Tensor, ctx: Context = None) -> torch.Tensor:
    g = torch.empty_like(x)
    _check(lib().lcs_gradient(_ctx(ctx), ctypes.byref(_mat(A, ctx)), _vec(x, A.n, name="x"), _ptr(g),
                              _stream()))
    return g


def spmv(A: Matrix, x: torch.Tensor, y: torch.Tensor, reps: int = 1, ctx: Context = None):
    prec = PREC_FP64 if x.dtype == torch.float64 else PREC_MIXED
    dt = torch.float64 if prec == PREC_FP64 else torch.float32
    _check(lib().lcs_spmv(_ctx(ctx), ctypes.byref(_mat(A, ctx)), _vec(x, A.n, dt, "x"), _vec(y, A.n, dt, "y"),
                          prec, int(reps), _stream()))
    return y


def gather_restricted(A: Matrix, idx: torch.Tensor, ctx: Context = None):
    """B = A[idx, idx] as (row_ptr int32[K+1], col int32[nnz], val float64[nnz])."""
    K = idx.numel()
    dev = A.device
    rp = torch.zeros(K + 1, dtype=torch.int32, device=dev)
    col = torch.empty(max(A.max_row * K, 1), dtype=torch.int32, device=dev)
    val = torch.empty(max(A.max_row * K, 1), dtype=torch.float64, device=dev)
    nnz = ctypes.c_int64(0)
    _check(lib().lcs_gather_restricted(_ctx(ctx), ctypes.byref(_mat(A, ctx)),
                                       _ptr(idx.contiguous()) if K else None, K, _ptr(rp), _ptr(col),
                                       _ptr(val), ctypes.byref(nnz), _stream()))
    return rp, col[:nnz.value], val[:nnz.value]


def gs_sweeps(A: Matrix, b: torch.Tensor, x: torch.Tensor, n_sweeps: int = 1, ctx: Context = None):
    _check(lib().lcs_gs_sweeps(_ctx(ctx), ctypes.byref(_mat(A, ctx)), _vec(b, A.n, name="b"),
                               _vec(x, A.n, name="x"), int(n_sweeps), _stream()))
    return x


def cast_coef(A: Matrix, ctx: Context = None) -> torch.Tensor:
    c32 = torch.empty(A.coef.shape, dtype=torch.float32, device=A.coef.device)
    _check(lib().lcs_cast_coef(_ctx(ctx), ctypes.byref(_mat(A, ctx)), _ptr(c32), _stream()))
    return c32


def assemble_logk(kind: int, nx: int, ny: int, nz: int, inv_dt: float, logk: torch.Tensor,
                  ctx: Context = None) -> torch.Tensor:
    n = nx * ny * nz
    coef = torch.empty((N_ARRAYS[kind], n), dtype=torch.float64, device=logk.device)
    _check(lib().lcs_assemble_logk(_ctx(ctx), kind, nx, ny, nz, float(inv_dt),
                                   _vec(logk.contiguous(), n, name="logk"), _ptr(coef), _stream()))
    return coef


def grad_logk(kind: int, nx: int, ny: int, nz: int, logk: torch.Tensor, x: torch.Tensor,
              lam: torch.Tensor, ctx: Context = None) -> torch.Tensor:
    n = nx * ny * nz
    g = torch.empty(n, dtype=torch.float64, device=x.device)
    _check(lib().lcs_grad_logk(_ctx(ctx), kind, nx, ny, nz, _vec(logk.contiguous(), n, name="logk"),
                               _vec(x, n, name="x"), _vec(lam, n, name="lam"), _ptr(g), _stream()))
    return g


def set_kernel_timing(what: int, ctx: Context = None):
    """Time one kernel class with HIP events (TIME_* constants); resets totals."""
    _check(lib().lcs_set_kernel_timing(_ctx(ctx), int(what)))


def get_kernel_timing(ctx: Context = None):
    """(total ms, number of timed launches) since the last set_kernel_timing."""
    ms = ctypes.c_double(0.0)
    n = ctypes.c_int64(0)
    _check(lib().lcs_get_kernel_timing(_ctx(ctx), ctypes.byref(ms), ctypes.byref(n)))
    return ms.value, n.value


def assemble_heat(nx: int, ny: int, inv_dt: float, power: float, t_left: float, t_right: float,
                  t_lin: torch.Tensor, t_old: torch.Tensor, coef: torch.Tensor = None,
                  b: torch.Tensor = None, ctx: Context = None):
    """Picard system of the 2-D heat-conduction test: (coef [3, N], b [N])."""
    n = nx * ny
    if coef is None:
        coef = torch.empty((3, n), dtype=torch.float64, device=t_lin.device)
    if b is None:
        b = torch.empty(n, dtype=torch.float64, device=t_lin.device)
    _check(lib().lcs_assemble_heat(_ctx(ctx), nx, ny, float(inv_dt), float(power), float(t_left),
                                   float(t_right), _vec(t_lin, n, name="t_lin"),
                                   _vec(t_old, n, name="t_old"), _vec(coef.view(-1), 3 * n, name="coef"),
                                   _vec(b, n, name="b"), _stream()))
    return coef, b


def norm2_diff(a: torch.Tensor, b: torch.Tensor, ctx: Context = None) -> float:
    """||a - b||_2 (FP64 device vectors of the same length)."""
    n = a.numel()
    out = ctypes.c_double(0.0)
    _check(lib().lcs_norm2_diff(_ctx(ctx), _vec(a, n, name="a"), _vec(b, n, name="b"), n,
                                ctypes.byref(out), _stream()))
    return out.value


def set_tiling(march_rows: int = 0, nontemporal: int = -1, ctx: Context = None):
    """Walk of the 2-D stencil kernels: march_rows < 0 flat, 0 automatic, > 0
    row-marching tiles of that many rows; nontemporal 0 turns the marching
    kernels' non-temporal hints off."""
    _check(lib().lcs_set_tiling(_ctx(ctx), int(march_rows), int(nontemporal)))


def set_colour_blocking(on: bool = True, ctx: Context = None):
    """Order of the restricted system's rows under RB-SGS: colour by colour
    (True, the default) or the domain's ascending order (False); per-row
    results are the same either way (lcs_set_colour_blocking)."""
    _check(lib().lcs_set_colour_blocking(_ctx(ctx), 1 if on else 0))


def set_short_columns(on: bool = True, ctx: Context = None):
    """Index form of the restricted system: columns coded per row where
    they fit (True, the default: the five- and nine-point stencils in grid
    order, and the red-black colour-blocked five- and seven-point rows under
    RB-SGS) or 32-bit indices (False); results are the same either way
    (lcs_set_short_columns)."""
    _check(lib().lcs_set_short_columns(_ctx(ctx), 1 if on else 0))


def matrix_from_numpy(kind: int, nx: int, ny: int, nz: int, coef, device="cuda",
                      with32: bool = False) -> Matrix:
    c = torch.as_tensor(coef, dtype=torch.float64).reshape(N_ARRAYS[kind], nx * ny * nz)
    c = c.to(device).contiguous()
    M = Matrix(kind, nx, ny, nz, c)
    if with32:
        M.coef32 = cast_coef(M)
    return M
