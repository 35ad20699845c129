"""Seeded synthetic inputs for the local character-based solver.

This module only *creates problems*: conductivity fields, the symmetric
stencil coefficients of the implicit diffusion operator, heat sources and the
right-hand side of each backward-Euler / Picard system.  It holds none of the
method's arithmetic (no residuals, no marking, no Krylov iteration), so the
HIP path and the CPU oracle can both consume its bytes without sharing code.

Operators (cell-centred finite volumes, h = 1, zero-flux outer faces):

* ``5pt`` (2-D) and ``7pt`` (3-D): A = I/dt + sum over faces f=(P,Q) of
  T_f (e_P - e_Q)(e_P - e_Q)^T with the harmonic face value
  T_f = 2 k_P k_Q / (k_P + k_Q), k = exp(log k).  This is the five-point
  scheme of the paper's 2-D heat test (Section 3.1) with backward Euler in
  time (its time-discrete equation), extended to 3-D.
* ``9pt`` (2-D): A = I/dt + sum over interior cell corners c of
  G_c^T K G_c, where G_c maps the four cells around the corner to a corner
  gradient and K is a constant rotated anisotropic tensor.  The sum is SPD
  but not an M-matrix (nine-point schemes are used for the paper's
  deformed-mesh radiation systems, Section 3.3).

Stencil storage is symmetric: ``coef[0]`` is the diagonal, the other rows hold
the coupling to the "forward" neighbours only (the backward ones are read from
the neighbour's entry).  Cell index i = x + nx*y (+ nx*ny*z).

  5pt : C, E=(+1,0), N=(0,+1)
  9pt : C, E=(+1,0), N=(0,+1), NE=(+1,+1), NW=(-1,+1)
  7pt : C, E=(+1,0,0), N=(0,+1,0), U=(0,0,+1)

Entries toward a neighbour outside the grid are 0 and are not part of the
sparsity pattern.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Callable, List, Optional

import numpy as np

KIND_5PT = 0
KIND_9PT = 1
KIND_7PT = 2
KIND_9N = 3       # nine-point, full storage (non-symmetric)
KIND_NAMES = {KIND_5PT: "5pt", KIND_9PT: "9pt", KIND_7PT: "7pt", KIND_9N: "9n"}
N_ARRAYS = {KIND_5PT: 3, KIND_9PT: 5, KIND_7PT: 4, KIND_9N: 9}

BASE_SEED = 20010115


# --------------------------------------------------------------------------
# conductivity fields and operators
# --------------------------------------------------------------------------
def lognormal_logk(shape, sigma: float, seed: int) -> np.ndarray:
    """Per-cell log-conductivity, i.i.d. N(0, sigma^2), from numpy's PCG64."""
    rng = np.random.default_rng(seed)
    return sigma * rng.standard_normal(size=shape)


def _harmonic(kp: np.ndarray, kq: np.ndarray) -> np.ndarray:
    return 2.0 * kp * kq / (kp + kq)


def assemble_5pt(logk: np.ndarray, inv_dt: float) -> np.ndarray:
    """Coefficients (3, N) of the 2-D five-point operator for logk[ny, nx]."""
    ny, nx = logk.shape
    k = np.exp(logk)
    tx = _harmonic(k[:, :-1], k[:, 1:])          # face between (x, y) and (x+1, y)
    ty = _harmonic(k[:-1, :], k[1:, :])          # face between (x, y) and (x, y+1)
    c = np.full((ny, nx), inv_dt)
    c[:, :-1] += tx
    c[:, 1:] += tx
    c[:-1, :] += ty
    c[1:, :] += ty
    e = np.zeros((ny, nx))
    e[:, :-1] = -tx
    n = np.zeros((ny, nx))
    n[:-1, :] = -ty
    return np.ascontiguousarray(np.stack([c, e, n]).reshape(3, nx * ny))


def assemble_7pt(logk: np.ndarray, inv_dt: float) -> np.ndarray:
    """Coefficients (4, N) of the 3-D seven-point operator for logk[nz, ny, nx]."""
    nz, ny, nx = logk.shape
    k = np.exp(logk)
    tx = _harmonic(k[:, :, :-1], k[:, :, 1:])
    ty = _harmonic(k[:, :-1, :], k[:, 1:, :])
    tz = _harmonic(k[:-1, :, :], k[1:, :, :])
    c = np.full((nz, ny, nx), inv_dt)
    c[:, :, :-1] += tx
    c[:, :, 1:] += tx
    c[:, :-1, :] += ty
    c[:, 1:, :] += ty
    c[:-1, :, :] += tz
    c[1:, :, :] += tz
    e = np.zeros((nz, ny, nx))
    e[:, :, :-1] = -tx
    n = np.zeros((nz, ny, nx))
    n[:, :-1, :] = -ty
    u = np.zeros((nz, ny, nx))
    u[:-1, :, :] = -tz
    return np.ascontiguousarray(np.stack([c, e, n, u]).reshape(4, nx * ny * nz))


def aniso_tensor(ratio: float, angle_deg: float):
    """K = R(angle) diag(1, 1/ratio) R(angle)^T as (kxx, kxy, kyy)."""
    t = math.radians(angle_deg)
    c, s = math.cos(t), math.sin(t)
    k1, k2 = 1.0, 1.0 / ratio
    return (c * c * k1 + s * s * k2, c * s * (k1 - k2), s * s * k1 + c * c * k2)


def assemble_9pt(nx: int, ny: int, inv_dt: float, ratio: float = 100.0,
                 angle_deg: float = 30.0) -> np.ndarray:
    """Coefficients (5, N) of the 2-D SPD nine-point anisotropic operator.

    Each interior corner c, shared by cells a=(x,y), b=(x+1,y), c=(x,y+1),
    d=(x+1,y+1), contributes G^T K G with the corner gradient
    gx = ((x_b - x_a) + (x_d - x_c))/2, gy = ((x_c - x_a) + (x_d - x_b))/2.
    """
    kxx, kxy, kyy = aniso_tensor(ratio, angle_deg)
    g = 0.5 * np.array([[-1.0, 1.0, -1.0, 1.0],
                        [-1.0, -1.0, 1.0, 1.0]])
    kt = np.array([[kxx, kxy], [kxy, kyy]])
    m = g.T @ kt @ g                                  # 4x4 local matrix, rows a,b,c,d
    off = [(0, 0), (1, 0), (0, 1), (1, 1)]            # cell offsets of a,b,c,d
    c = np.full((ny, nx), inv_dt)
    e = np.zeros((ny, nx))
    n = np.zeros((ny, nx))
    ne = np.zeros((ny, nx))
    nw = np.zeros((ny, nx))
    cy, cx = ny - 1, nx - 1                           # interior corners
    for p in range(4):
        px, py = off[p]
        c[py:py + cy, px:px + cx] += m[p, p]
        for q in range(4):
            if q == p:
                continue
            dx, dy = off[q][0] - px, off[q][1] - py
            # keep only forward couplings; the others are their transposes
            if (dx, dy) == (1, 0):
                e[py:py + cy, px:px + cx] += m[p, q]
            elif (dx, dy) == (0, 1):
                n[py:py + cy, px:px + cx] += m[p, q]
            elif (dx, dy) == (1, 1):
                ne[py:py + cy, px:px + cx] += m[p, q]
            elif (dx, dy) == (-1, 1):
                nw[py:py + cy, px:px + cx] += m[p, q]
    return np.ascontiguousarray(np.stack([c, e, n, ne, nw]).reshape(5, nx * ny))


# --------------------------------------------------------------------------
# sources
# --------------------------------------------------------------------------
def disk_source(nx: int, ny: int, cx: float, cy: float, radius: float, q: float) -> np.ndarray:
    y, x = np.mgrid[0:ny, 0:nx]
    return np.where((x - cx) ** 2 + (y - cy) ** 2 <= radius * radius, q, 0.0).reshape(-1)


def ball_source(nx: int, ny: int, nz: int, cx: float, cy: float, cz: float,
                radius: float, q: float) -> np.ndarray:
    z, y, x = np.mgrid[0:nz, 0:ny, 0:nx]
    r2 = (x - cx) ** 2 + (y - cy) ** 2 + (z - cz) ** 2
    return np.where(r2 <= radius * radius, q, 0.0).reshape(-1)


def patch_mask(nx: int, ny: int, x0: int, y0: int, w: int) -> np.ndarray:
    m = np.zeros((ny, nx))
    m[y0:y0 + w, x0:x0 + w] = 1.0
    return m.reshape(-1)


# --------------------------------------------------------------------------
# system sequences
# --------------------------------------------------------------------------
@dataclasses.dataclass
class Workload:
    """A sequence of SPD systems A x_k = b_k sharing one operator A.

    ``rhs(k, x_prev)`` gives b_k from the previous solution (backward Euler:
    b_k = x_prev/dt + q_k; Picard: b_s = x_n/dt + q(x_s)).  ``x_start`` is
    the initial state x_{-1}.  Threshold and solver settings are part of the
    workload because the configurations name them.
    """
    name: str
    kind: int
    nx: int
    ny: int
    nz: int
    dt: float
    coef: np.ndarray            # (n_arrays, N) float64
    n_systems: int
    rhs: Callable[[int, np.ndarray], np.ndarray]
    x_start: np.ndarray
    logk: Optional[np.ndarray] = None
    eps: float = 1e-10
    theta_res: float = 1e-3
    alpha_grad: float = 1e-4
    e_max: int = 1
    precision: str = "fp64"     # or "mixed"
    precond: str = "jacobi"     # or "rbsgs"
    notes: str = ""

    @property
    def n(self) -> int:
        return self.nx * self.ny * self.nz

    @property
    def dims(self):
        return (self.nx, self.ny, self.nz)


def c1_picard(nx: int = 64, ny: int = 64, sigma: float = 0.5, dt: float = 4.0,
              patch: int = 8, q0: float = 1.0, n_systems: int = 10,
              seed: int = BASE_SEED + 0) -> Workload:
    """2-D nonlinear heat step: Picard iterates of A T_{s+1} = T_n/dt + q(T_s),
    q(T) = q0 * 1_patch / (1 + T) on a patch x patch hot spot at the centre.
    Only the patch entries of b change between systems."""
    logk = lognormal_logk((ny, nx), sigma, seed)
    inv_dt = 1.0 / dt
    coef = assemble_5pt(logk, inv_dt)
    pm = patch_mask(nx, ny, (nx - patch) // 2, (ny - patch) // 2, patch)
    t_n = np.zeros(nx * ny)

    def rhs(k: int, x_prev: np.ndarray) -> np.ndarray:
        return t_n * inv_dt + q0 * pm / (1.0 + x_prev)

    return Workload("c1_picard_64x64_5pt", KIND_5PT, nx, ny, 1, dt, coef, n_systems,
                    rhs, t_n.copy(), logk, theta_res=1e-3, e_max=1,
                    notes="Picard sequence, 8x8 nonlinear source patch")


def c2_moving_disk(nx: int = 1024, ny: int = 1024, sigma: float = 1.0, dt: float = 4.0,
                   radius: float = 40.0, speed: float = 4.0, q0: float = 1.0,
                   n_systems: int = 20, seed: int = BASE_SEED + 1,
                   x_offset: Optional[float] = None) -> Workload:
    """2-D backward-Euler sequence with a disk heat source moving in +x."""
    logk = lognormal_logk((ny, nx), sigma, seed)
    inv_dt = 1.0 / dt
    coef = assemble_5pt(logk, inv_dt)
    x0c = nx / 4.0 if x_offset is None else x_offset

    def rhs(k: int, x_prev: np.ndarray) -> np.ndarray:
        q = disk_source(nx, ny, x0c + speed * k, ny / 2.0, radius, q0)
        return x_prev * inv_dt + q

    return Workload(f"c2_moving_disk_{nx}x{ny}_5pt", KIND_5PT, nx, ny, 1, dt, coef, n_systems,
                    rhs, np.zeros(nx * ny), logk, theta_res=1e-3, alpha_grad=1e-4, e_max=1)


def c3_aniso_front(nx: int = 4096, ny: int = 4096, dt: float = 4.0, ratio: float = 100.0,
                   angle: float = 30.0, radius: float = 350.0, speed: float = 8.0,
                   q0: float = 1.0, n_systems: int = 20) -> Workload:
    """2-D nine-point rotated anisotropic operator, moving disk front.  With
    radius 350 the changing region (disk plus a ~40-cell tail) covers about
    3 % of a 4096^2 grid under the paper's residual threshold."""
    inv_dt = 1.0 / dt
    coef = assemble_9pt(nx, ny, inv_dt, ratio, angle)
    x0c = nx / 4.0

    def rhs(k: int, x_prev: np.ndarray) -> np.ndarray:
        q = disk_source(nx, ny, x0c + speed * k, ny / 2.0, radius, q0)
        return x_prev * inv_dt + q

    return Workload(f"c3_aniso9_{nx}x{ny}", KIND_9PT, nx, ny, 1, dt, coef, n_systems,
                    rhs, np.zeros(nx * ny), None, theta_res=1e-3, e_max=1,
                    precision="mixed", precond="jacobi")


def full_from_symmetric9(nx: int, ny: int, sym: np.ndarray) -> np.ndarray:
    """Full storage (9, N) of a symmetric nine-point operator given in
    symmetric storage (C, E, N, NE, NW): slot s of row i holds a(i, j_s) for
    the neighbours SW, S, SE, W, C, E, NW, N, NE; zero outside the grid."""
    c, e, nn, ne, nw = (np.asarray(a).reshape(ny, nx) for a in sym)
    f = np.zeros((9, ny, nx))
    f[0][1:, 1:] = ne[:-1, :-1]        # SW: the NE coupling of (x-1, y-1)
    f[1][1:, :] = nn[:-1, :]           # S
    f[2][1:, :-1] = nw[:-1, 1:]        # SE: the NW coupling of (x+1, y-1)
    f[3][:, 1:] = e[:, :-1]            # W
    f[4] = c
    f[5][:, :-1] = e[:, :-1]           # E
    f[6][:-1, 1:] = nw[:-1, 1:]        # NW
    f[7][:-1, :] = nn[:-1, :]          # N
    f[8][:-1, :-1] = ne[:-1, :-1]      # NE
    return f.reshape(9, nx * ny)


def assemble_9n(nx: int, ny: int, inv_dt: float, ratio: float = 4.0, angle_deg: float = 30.0,
                speed: float = 2.0) -> np.ndarray:
    """Full-storage coefficients (9, N) of a non-symmetric nine-point
    operator: the symmetric corner-gradient diffusion of assemble_9pt plus
    first-order upwind convection by the rotating, divergence-free velocity
    u = speed * (-(y - cy), x - cx) / (n / 2) (cells of size 1), standing in
    for the convection-bearing schemes on deforming meshes of the paper's
    application.  Face velocities are sampled at face centres; each face
    adds max(u_f, 0) to the upwind cell's diagonal and min(u_f, 0) to its
    coupling to the downwind cell."""
    f = full_from_symmetric9(nx, ny, assemble_9pt(nx, ny, inv_dt, ratio, angle_deg))
    f = f.reshape(9, ny, nx)
    scale = speed / (0.5 * max(nx, ny))
    cx, cy = nx / 2.0, ny / 2.0
    y, x = np.mgrid[0:ny, 0:nx].astype(np.float64)
    ue = -scale * ((y + 0.5) - cy)          # x-velocity at the east face of each cell
    vn = scale * ((x + 0.5) - cx)           # y-velocity at the north face of each cell
    # east faces between (x, y) and (x+1, y)
    a = ue[:, :-1]
    f[4][:, :-1] += np.maximum(a, 0.0)
    f[5][:, :-1] += np.minimum(a, 0.0)
    f[4][:, 1:] += np.maximum(-a, 0.0)
    f[3][:, 1:] += np.minimum(-a, 0.0)
    # north faces between (x, y) and (x, y+1)
    v = vn[:-1, :]
    f[4][:-1, :] += np.maximum(v, 0.0)
    f[7][:-1, :] += np.minimum(v, 0.0)
    f[4][1:, :] += np.maximum(-v, 0.0)
    f[1][1:, :] += np.minimum(-v, 0.0)
    return np.ascontiguousarray(f.reshape(9, nx * ny))


def c6_nonsym9(nx: int = 1024, ny: int = 1024, dt: float = 4.0, radius: float = 40.0,
               speed: float = 4.0, q0: float = 1.0, n_systems: int = 20) -> Workload:
    """2-D non-symmetric nine-point sequence (diffusion with anisotropy 4 at
    30 degrees plus upwind convection in a rotating flow), disk source moving
    `speed` cells per system; solved by GMRES(40)."""
    inv_dt = 1.0 / dt
    coef = assemble_9n(nx, ny, inv_dt)
    x0c = nx / 4.0

    def rhs(k: int, x_prev: np.ndarray) -> np.ndarray:
        q = disk_source(nx, ny, x0c + speed * k, ny / 2.0, radius, q0)
        return x_prev * inv_dt + q

    return Workload(f"c6_nonsym9_{nx}x{ny}", KIND_9N, nx, ny, 1, dt, coef, n_systems,
                    rhs, np.zeros(nx * ny), None, theta_res=1e-3, e_max=1,
                    precision="fp64", precond="jacobi")


def c4_adjoint(nx: int = 2048, ny: int = 2048, sigma: float = 1.0, dt: float = 4.0,
               radius: float = 40.0, speed: float = 4.0, window: int = 256,
               k_sys: int = 10, seed: int = BASE_SEED + 3) -> Workload:
    """2-D five-point FP64 system used for the adjoint (loss over a window)."""
    w = c2_moving_disk(nx, ny, sigma, dt, radius, speed, 1.0, k_sys + 1, seed,
                       x_offset=nx / 2.0 - speed * k_sys)
    w.name = f"c4_adjoint_{nx}x{ny}_5pt"
    w.notes = f"loss window {window}x{window} centred on the front at system {k_sys}"
    return w


def c5_sphere3d(n: int = 256, sigma: float = 1.5, dt: float = 4.0, radius: float = 20.0,
                speed: float = 2.0, q0: float = 1.0, n_systems: int = 50,
                seed: int = BASE_SEED + 4) -> Workload:
    """3-D seven-point sequence with a spherical source moving in +x."""
    logk = lognormal_logk((n, n, n), sigma, seed)
    inv_dt = 1.0 / dt
    coef = assemble_7pt(logk, inv_dt)
    x0c = n / 4.0

    def rhs(k: int, x_prev: np.ndarray) -> np.ndarray:
        q = ball_source(n, n, n, x0c + speed * k, n / 2.0, n / 2.0, radius, q0)
        return x_prev * inv_dt + q

    return Workload(f"c5_sphere_{n}^3_7pt", KIND_7PT, n, n, n, dt, coef, n_systems,
                    rhs, np.zeros(n ** 3), logk, theta_res=1e-3, e_max=1,
                    precision="mixed", precond="rbsgs")


# --------------------------------------------------------------------------
# worked example of the paper (Example 1, Section 2.3)
# --------------------------------------------------------------------------
def example1():
    """The 9x9 tridiagonal system of the paper's Example 1 as dense arrays.

    a_ii = 1, a_{i,i+1} = a_{i+1,i} = -1/(i+2) for 0-based i; the exact
    solution is x_i = 10^-(i+1); the initial iterate is 1, 0.1, then
    1.001 * 10^-(i+1).  b = A x.  Returns (A, x, x0, b).
    """
    nn = 9
    a = np.eye(nn)
    for i in range(nn - 1):
        a[i, i + 1] = a[i + 1, i] = -1.0 / (i + 2)
    x = np.array([10.0 ** -(i + 1) for i in range(nn)])
    x0 = np.array([1.0, 1e-1] + [1.001 * 10.0 ** -(i + 1) for i in range(2, nn)])
    b = a @ x
    return a, x, x0, b


# ---------------------------------------------------------------------------
# 2-D nonlinear heat-conduction test problem (Section 3.1)
# ---------------------------------------------------------------------------
HEAT_T_LEFT = 1.0          # T at x = 0
HEAT_T_RIGHT = 1e-4        # T at x = 1
HEAT_POWER = 3.5           # k(T) = T^3.5
HEAT_DT = 1e-2             # time step
HEAT_STEPS = 100           # physical time 0 .. 1
HEAT_PICARD_TOL = 1e-8     # ||T^(n+1,s+1) - T^(n+1,s)||_2
HEAT_ALPHA = 1e-4          # gradient threshold of the gradient-based method
HEAT_E_MAX = 1             # expansion rounds of the residual-based method


def heat2d_initial(nx: int, ny: int) -> np.ndarray:
    """T_0(x, y) = exp(-100 x) T_l + T_r at the centres of nx x ny cells of the
    unit square, row-major (y slowest)."""
    x = (np.arange(nx) + 0.5) / nx
    return np.ascontiguousarray(np.tile(np.exp(-100.0 * x) * HEAT_T_LEFT + HEAT_T_RIGHT, ny))


# ---------------------------------------------------------------------------
# Multi-group batch (Section 3.3, Algorithm 7): G decoupled group systems
# ---------------------------------------------------------------------------
MG_EPS = 1e-8              # linear tolerance of the paper's multi-group test
MG_ALPHA = 1e-10           # gradient threshold of the gradient-based method there
MG_E_MAX = 1


@dataclasses.dataclass
class MGBatch:
    name: str
    nx: int
    ny: int
    G: int
    coef: np.ndarray       # (G, 5, N) nine-point operators
    b: np.ndarray          # (G, N)
    x0: np.ndarray         # (G, N) previous state of each group
    kappa: np.ndarray      # (G,) diffusion coefficient per group
    kind: int = KIND_9PT   # KIND_9PT (coef (G, 5, N)) or KIND_9N (coef (G, 9, N))


def _scipy_matrix(kind: int, nx: int, ny: int, nz: int, coef: np.ndarray):
    """The full symmetric matrix of a stencil coefficient set (scipy CSR), to
    generate previous states by a direct solve."""
    import scipy.sparse as sp
    n = nx * ny * nz
    c = np.asarray(coef).reshape(N_ARRAYS[kind], n)
    idx = np.arange(n).reshape(nz, ny, nx)
    rows, cols, vals = [np.arange(n)], [np.arange(n)], [c[0]]

    def couple(arr, src, dst):
        rows.extend([src, dst])
        cols.extend([dst, src])
        vals.extend([arr[src], arr[src]])

    couple(c[1], idx[:, :, :-1].ravel(), idx[:, :, 1:].ravel())            # E
    couple(c[2], idx[:, :-1, :].ravel(), idx[:, 1:, :].ravel())            # N
    if kind == KIND_9PT:
        couple(c[3], idx[:, :-1, :-1].ravel(), idx[:, 1:, 1:].ravel())     # NE
        couple(c[4], idx[:, :-1, 1:].ravel(), idx[:, 1:, :-1].ravel())     # NW
    if kind == KIND_7PT:
        couple(c[3], idx[:-1].ravel(), idx[1:].ravel())                    # U
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(n, n))


def mg_batch(nx: int = 88, ny: int = 80, G: int = 64, dt: float = 1.0, sigma: float = 1.0,
             kappa_lo: float = 0.1, kappa_hi: float = 316.0, radius: float = 6.0,
             shift: float = 3.0, seed: int = BASE_SEED + 6) -> MGBatch:
    """The G group systems of one source iteration: nx x ny = 7040 cells (the
    paper's cell count), nine-point operators (anisotropy 4 at 30 degrees,
    standing in for a deforming mesh), A_g = (1/dt + sigma) I + kappa_g L with
    kappa_g log-spaced from kappa_lo to kappa_hi (higher groups diffuse
    further, so their local domains grow, as the paper reports).

    x0_g is the steady state of a disk source of strength Q_g (log-normal per
    group) at c0: (sigma I + kappa_g L) x0_g = q(c0).  The new system has the
    disk moved by `shift` cells: b_g = x0_g / dt + q(c1), so
    A_g (x_g - x0_g) = q(c1) - q(c0): the change is driven by the source's
    move alone and spreads over sqrt(kappa_g / (1/dt + sigma)) cells."""
    import scipy.sparse.linalg as spla
    rng = np.random.default_rng(seed)
    n = nx * ny
    kappa = np.exp(np.linspace(np.log(kappa_lo), np.log(kappa_hi), G))
    qg = np.exp(rng.normal(0.0, 0.5, G))
    lap = assemble_9pt(nx, ny, 0.0, 4.0, 30.0)          # L alone (zero mass)
    c0 = (nx / 2.0 - shift / 2.0, ny / 2.0)
    c1 = (nx / 2.0 + shift / 2.0, ny / 2.0)
    coef = np.empty((G, 5, n))
    b = np.empty((G, n))
    x0 = np.empty((G, n))
    for g in range(G):
        L = kappa[g] * lap
        ss = L.copy()
        ss[0] += sigma
        q0 = disk_source(nx, ny, c0[0], c0[1], radius, qg[g])
        q1 = disk_source(nx, ny, c1[0], c1[1], radius, qg[g])
        x0[g] = spla.spsolve(_scipy_matrix(KIND_9PT, nx, ny, 1, ss).tocsc(), q0)
        coef[g] = L
        coef[g, 0] += 1.0 / dt + sigma
        b[g] = x0[g] / dt + q1
    return MGBatch(f"mg{G}_{nx}x{ny}_9pt", nx, ny, G, coef, b, x0, kappa)


NINE_OFFSETS = [(-1, -1), (-1, 0), (-1, 1), (0, -1), (0, 0), (0, 1), (1, -1), (1, 0), (1, 1)]


def _scipy_matrix_9n(nx: int, ny: int, coef: np.ndarray):
    """The matrix of full-storage nine-point coefficients (scipy CSR): slot k
    of row (x, y) couples to (x + dx_k, y + dy_k), in the slot order of
    assemble_9n, to generate previous states by a direct solve."""
    import scipy.sparse as sp
    c = np.asarray(coef).reshape(9, ny, nx)
    y, x = np.mgrid[0:ny, 0:nx]
    rows, cols, vals = [], [], []
    for k, (dy, dx) in enumerate(NINE_OFFSETS):
        m = (x + dx >= 0) & (x + dx < nx) & (y + dy >= 0) & (y + dy < ny)
        rows.append((y * nx + x)[m])
        cols.append(((y + dy) * nx + (x + dx))[m])
        vals.append(c[k][m])
    n = nx * ny
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(n, n))


def mg_batch_nonsym(nx: int = 88, ny: int = 80, G: int = 64, dt: float = 1.0, sigma: float = 1.0,
                    kappa_lo: float = 0.1, kappa_hi: float = 316.0, radius: float = 6.0,
                    shift: float = 3.0, speed: float = 2.0,
                    seed: int = BASE_SEED + 7) -> MGBatch:
    """The G group systems of mg_batch with non-symmetric operators, as the
    paper's deforming-mesh systems are (solved by GMRES):
    A_g = (1/dt + sigma) I + kappa_g D + C, with D the anisotropic nine-point
    diffusion of assemble_9n and C its upwind convection in a rotating flow of
    the given speed, the same for every group.  x0_g is the steady state of the
    source at c0, (sigma I + kappa_g D + C) x0_g = q(c0), and b_g moves the
    source to c1, as in mg_batch."""
    import scipy.sparse.linalg as spla
    rng = np.random.default_rng(seed)
    n = nx * ny
    kappa = np.exp(np.linspace(np.log(kappa_lo), np.log(kappa_hi), G))
    qg = np.exp(rng.normal(0.0, 0.5, G))
    dif = assemble_9n(nx, ny, 0.0, 4.0, 30.0, speed=0.0)
    conv = assemble_9n(nx, ny, 0.0, 4.0, 30.0, speed=speed) - dif
    c0 = (nx / 2.0 - shift / 2.0, ny / 2.0)
    c1 = (nx / 2.0 + shift / 2.0, ny / 2.0)
    coef = np.empty((G, 9, n))
    b = np.empty((G, n))
    x0 = np.empty((G, n))
    for g in range(G):
        L = kappa[g] * dif + conv
        ss = L.copy()
        ss[4] += sigma
        q0 = disk_source(nx, ny, c0[0], c0[1], radius, qg[g])
        q1 = disk_source(nx, ny, c1[0], c1[1], radius, qg[g])
        x0[g] = spla.spsolve(_scipy_matrix_9n(nx, ny, ss).tocsc(), q0)
        coef[g] = L
        coef[g, 4] += 1.0 / dt + sigma
        b[g] = x0[g] / dt + q1
    return MGBatch(f"mg{G}_{nx}x{ny}_9n", nx, ny, G, coef, b, x0, kappa, kind=KIND_9N)


# ---------------------------------------------------------------------------
# General sparse input: an irregular graph over the cells of an nx x ny grid
# ---------------------------------------------------------------------------
def irregular_spd(nx: int, ny: int, seed: int, p_diag: float = 0.5, p_long: float = 0.1,
                  sigma: float = 1.0, mass: float = 0.25, hub_every: int = 0,
                  hub_len: tuple = (17, 64)):
    """Symmetric, strictly diagonally dominant M-matrix on an irregular graph
    (a stand-in for an unstructured mesh): every cell couples to its four
    grid neighbours, to each diagonal neighbour with probability p_diag and
    to the cell two steps east or north with probability p_long, with
    log-normal weights; the diagonal is the sum of the weights plus mass.
    At most 11 entries per row.  With hub_every > 0, every hub_every-th cell
    is a hub linked to random distant cells until its row holds a length
    drawn from hub_len (rows of 17 to 64 entries, as around a vertex of high
    degree), and no other row grows past 16 entries.  Returns CSR (rp int64,
    col int32 ascending, val float64)."""
    rng = np.random.default_rng(seed)
    n = nx * ny
    rows = [dict() for _ in range(n)]

    def link(i, j):
        w = math.exp(sigma * rng.standard_normal())
        rows[i][j] = -w
        rows[j][i] = -w

    for y in range(ny):
        for x in range(nx):
            i = x + nx * y
            if x + 1 < nx:
                link(i, i + 1)
            if y + 1 < ny:
                link(i, i + nx)
            if x + 1 < nx and y + 1 < ny and rng.random() < p_diag:
                link(i, i + nx + 1)
            if x > 0 and y + 1 < ny and rng.random() < p_diag:
                link(i, i + nx - 1)
            if x + 2 < nx and rng.random() < p_long:
                link(i, i + 2)
            if y + 2 < ny and rng.random() < p_long:
                link(i, i + 2 * nx)
    if hub_every > 0:
        hubs = set(range(hub_every // 2, n, hub_every))
        for h in sorted(hubs):
            want = int(rng.integers(hub_len[0], hub_len[1] + 1)) - 1   # entries besides the diagonal
            tries = 0
            while len(rows[h]) < want and tries < 50 * want:
                tries += 1
                j = int(rng.integers(0, n))
                if j == h or j in rows[h] or j in hubs or len(rows[j]) >= 15:
                    continue
                link(h, j)
    rp = np.zeros(n + 1, np.int64)
    cols, vals = [], []
    for i in range(n):
        r = rows[i]
        r[i] = -sum(r.values()) + mass
        for j in sorted(r):
            cols.append(j)
            vals.append(r[j])
        rp[i + 1] = len(cols)
    return rp, np.array(cols, np.int32), np.array(vals, np.float64)


def greedy_colouring(rp: np.ndarray, col: np.ndarray):
    """Colour rows in index order with the smallest colour unused by any
    stored neighbour (no entry joins two rows of one colour).  Returns
    (colour int8[n], number of colours)."""
    n = rp.size - 1
    colour = np.full(n, -1, np.int64)
    for i in range(n):
        used = {int(colour[j]) for j in col[rp[i]:rp[i + 1]] if j != i and colour[j] >= 0}
        c = 0
        while c in used:
            c += 1
        colour[i] = c
    return colour.astype(np.int8), int(colour.max()) + 1 if n else 0


def irregular_nonsym(nx: int, ny: int, seed: int, skew: float = 0.6, mass: float = 0.25, **kw):
    """Non-symmetric variant of irregular_spd (a convection-like skew): each
    coupling pair i < j gets a_ij = -w (1 + s), a_ji = -w (1 - s) with s
    uniform in [-skew, skew]; the diagonal is the row's absolute off-diagonal
    sum plus mass, so every row is strictly diagonally dominant.  Same
    pattern as irregular_spd(nx, ny, seed, **kw)."""
    rp, col, val = irregular_spd(nx, ny, seed, mass=mass, **kw)
    rng = np.random.default_rng(seed + 1000)
    n = rp.size - 1
    pos = {}
    for i in range(n):
        for k in range(rp[i], rp[i + 1]):
            pos[(i, int(col[k]))] = k
    val = val.copy()
    for i in range(n):
        for k in range(rp[i], rp[i + 1]):
            j = int(col[k])
            if j > i:
                s = rng.uniform(-skew, skew)
                val[k] *= 1.0 + s
                val[pos[(j, i)]] *= 1.0 - s
    for i in range(n):
        off = [k for k in range(rp[i], rp[i + 1]) if col[k] != i]
        val[pos[(i, i)]] = sum(abs(val[k]) for k in off) + mass
    return rp, col, val
