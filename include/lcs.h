/*
 * lcs.h -- C ABI of the MI355X (gfx950) local character-based solver.
 *
 * Method: Ye, An, Xu, "A local character based method for solving linear
 * systems of radiation diffusion problems" (arXiv 2001.01158).  For a system
 * A x = b whose initial iterate x^(0) is the previous time step or nonlinear
 * iterate (Section 2.1), the library
 *   1. marks a local domain Omega by residual (Section 2.3, Algorithm 3) or by
 *      the gradient mimic (Section 2.2, eq. grad, Algorithm 2),
 *   2. compacts Omega into the restricted CSR system B = A[Omega, Omega]
 *      (eq. BEFC) and solves B x_B = b_B - E x_C^(0) (eq. loc-equ) with PCG,
 *   3. assembles x~ (eq. sol-assemble), applies Gauss-Seidel smoothing, and
 *      finishes with a warm-started global PCG when x~ misses the criterion
 *      ||b - A x|| <= eps ||b|| (eq. rel-res-conv-criteria; Algorithm 1).
 *
 * Conventions shared by every entry point
 *   - Matrices are symmetric stencils on a structured grid, row index
 *     i = x + nx*y (+ nx*ny*z).  coef is a device array of n_arrays x N
 *     doubles: row 0 the diagonal, then the couplings to forward neighbours
 *       5-point 2-D : C, E(+1,0), N(0,+1)                        (3 arrays)
 *       9-point 2-D : C, E(+1,0), N(0,+1), NE(+1,+1), NW(-1,+1)   (5 arrays)
 *       7-point 3-D : C, E(+1,0,0), N(0,+1,0), U(0,0,+1)          (4 arrays)
 *     a backward coupling is the forward coupling stored at the neighbour.
 *     The sparsity pattern is every in-grid stencil neighbour.
 *   - LCS_STENCIL9N_2D is the non-symmetric nine-point operator (for example
 *     a deforming-mesh scheme with convection, Section 3.3) in full storage:
 *     9 arrays, array s holding each row's own coefficient at slot s, slots
 *     in ascending column order SW(-1,-1), S(0,-1), SE(+1,-1), W(-1,0), C,
 *     E(+1,0), NW(-1,+1), N(0,+1), NE(+1,+1); entries whose neighbour lies
 *     outside the grid are ignored.  Its solves (global, local, and the
 *     global finish) use restarted GMRES(m), the paper's Krylov method,
 *     right-preconditioned by Jacobi or nothing, in FP64; the criterion and
 *     Algorithm 1 are unchanged.  Batched solves and the adjoint take the
 *     symmetric kinds only.
 *   - LCS_CSR is a general sparse matrix (the paper's setting before any
 *     grid is assumed, Section 2.1) in CSR, symmetric unless csr_nonsym is
 *     set (then solved by GMRES(m) as LCS_STENCIL9N_2D is): nx = N, ny = nz = 1,
 *     row_ptr int32[N+1], col int32[nnz] strictly ascending within each row
 *     with the diagonal stored, val double[nnz]; every row holds 1..64
 *     entries.  Each call checks this structure before any kernel reads
 *     through col (LCS_EINVAL naming what failed; symmetry is the caller's
 *     to ensure, as for the stencils) and copies A into column-major ELL
 *     of width 5, 7, 9, 16 or 64 in the context's workspace, on which the whole path
 *     runs.  Scores, thresholds, expansion, compaction and the gather of B
 *     follow the stencil kinds' definitions over the stored entries.  The
 *     Gauss-Seidel sweeps and the RB-SGS preconditioner need a colouring:
 *     colour uint8[N] (device) with n_colours classes such that no stored
 *     off-diagonal entry joins two rows of one colour (checked).  Without
 *     one (colour = NULL) Algorithm 1 skips the smoothing step, RB-SGS and
 *     lcs_gs_sweeps return LCS_EINVAL.  coef and coef32 are ignored; the
 *     FP32 copy for LCS_PREC_MIXED is made inside each call.  Batched
 *     solves, lcs_cast_coef and the adjoint helpers take stencils only.
 *   - Vector arguments are device pointers of length N = nx*ny*nz (FP64)
 *     owned by the caller; the library never frees them.  Index arrays are
 *     int32 (N < 2^31).
 *   - stream is a hipStream_t (NULL = default stream).  Work is enqueued on
 *     it; calls that need a host decision (K, convergence) synchronise it
 *     before returning.
 *   - Every call returns an lcs_status; on error lcs_last_error() gives a
 *     message (thread-local).  No exception crosses the ABI.  On
 *     LCS_ENOCONV / LCS_EBREAKDOWN, x holds the last iterate and stats are
 *     filled.
 *   - A context made by lcs_create owns its device workspace (hipMalloc'd,
 *     grown on demand, released by lcs_destroy; growing it synchronises the
 *     device).  A context made by lcs_create_with_workspace takes every
 *     device buffer from one caller-owned buffer and never allocates,
 *     frees or synchronises the device in a call.  A context is used by one
 *     host thread at a time; calls on one context serialise on its
 *     workspace.
 */
#ifndef LCS_H
#define LCS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum lcs_status {
    LCS_OK = 0,
    LCS_EINVAL = 1,       /* bad argument (sizes, kinds, NULL pointers)          */
    LCS_EHIP = 2,         /* a HIP runtime call failed                            */
    LCS_ENOMEM = 3,       /* device workspace allocation failed                   */
    LCS_ENOCONV = 4,      /* max_iter / max_outer reached before the criterion    */
    LCS_EBREAKDOWN = 5,   /* p^T A p <= 0 in CG: the operator is not SPD          */
    LCS_ENONFINITE = 6    /* NaN / Inf in the input or the iteration              */
} lcs_status;

enum { LCS_STENCIL5_2D = 0, LCS_STENCIL9_2D = 1, LCS_STENCIL7_3D = 2, LCS_STENCIL9N_2D = 3,
       LCS_CSR = 4 };
enum { LCS_MODE_RESIDUAL = 0, LCS_MODE_GRADIENT = 1 };
enum {
    LCS_THRESH_REL_MAX = 0,  /* tau = theta * max_i |s_i|  (s = r^(0) or g)       */
    LCS_THRESH_ABS = 1,      /* tau = theta                                        */
    LCS_THRESH_PAPER = 2     /* tau = theta * ||b||_2 / sqrt(N), theta = epsilon,
                                eq. (resi-local-domain-0); residual mode only      */
};
enum { LCS_PC_NONE = 0, LCS_PC_JACOBI = 1, LCS_PC_RBSGS = 2 };
enum { LCS_PREC_FP64 = 0, LCS_PREC_MIXED = 1 };

typedef struct lcs_matrix {
    int32_t kind;          /* LCS_STENCIL* or LCS_CSR                              */
    int32_t nx, ny, nz;    /* grid; nz = 1 in 2-D; CSR: N, 1, 1                    */
    const double *coef;    /* device, n_arrays x N, FP64                           */
    const float *coef32;   /* device, n_arrays x N, FP32 copy for LCS_PREC_MIXED;
                              NULL: the library casts coef into its workspace      */
    /* LCS_CSR only (zero / NULL for the stencil kinds) */
    const int32_t *row_ptr;   /* device, N + 1                                     */
    const int32_t *col;       /* device, nnz                                       */
    const double *val;        /* device, nnz                                       */
    int64_t nnz;
    const uint8_t *colour;    /* device, N, or NULL                                */
    int32_t n_colours;        /* 1..255 with a colouring                           */
    int32_t csr_reuse;        /* 1: the caller states that these arrays, at these
                                 addresses, are unchanged since the previous call
                                 on this context that checked and copied them;
                                 the context then reuses its ELL copy (pointers,
                                 N, nnz and n_colours must match, else the call
                                 checks and copies as with 0).  The library cannot
                                 see values edited in place, nor a new matrix of
                                 the same shape placed at the freed addresses of
                                 the old one (as a caching allocator may do): set
                                 1 only for arrays known to be unchanged        */
    int32_t csr_nonsym;       /* 1: A is not symmetric; every solve (global,
                                 local, global finish) uses GMRES(m) in FP64
                                 with Jacobi or no preconditioner, as for
                                 LCS_STENCIL9N_2D                                */
} lcs_matrix;

typedef struct lcs_options {
    double eps;            /* global criterion ||b - A x||_2 <= eps ||b||_2 (1e-10) */
    double tol_local;      /* local criterion ||r_B||_2 <= tol_local ||b||_2;
                              <= 0 means eps                                        */
    double inner_tol;      /* mixed precision: inner FP32 PCG stops at
                              ||r32|| <= inner_tol ||r32_0|| (default 1e-5)         */
    int32_t max_iter;      /* PCG iteration cap per solve (all outer steps)         */
    int32_t precond;       /* LCS_PC_*; RBSGS is the symmetric colour-ordered
                              Gauss-Seidel preconditioner from z = 0 (colours
                              0..c-1, then back to 0): red-black (c = 2) for the
                              5- and 7-point stencils, four colours (x mod 2 +
                              2 (y mod 2)) for the 9-point stencil; EINVAL for
                              LCS_STENCIL9N_2D                                      */
    int32_t precision;     /* LCS_PREC_FP64 or LCS_PREC_MIXED                       */
    int32_t n_smooth;      /* Gauss-Seidel sweeps on x~ (Algorithm 1 step 7)        */
    int32_t check_every;   /* PCG iterations between host convergence checks       */
    int32_t max_outer;     /* mixed: refinement steps; FP64: restarts after a
                              failed true-residual check                            */
    int32_t restart;       /* GMRES restart length m (LCS_STENCIL9N_2D), 1..64;
                              default 40                                            */
} lcs_options;

typedef struct lcs_stats {
    int64_t K;             /* |Omega|                                               */
    int32_t e_rounds;      /* expansion rounds that added points                   */
    int32_t its_local;     /* PCG iterations on B (all refinement steps)            */
    int32_t its_global;    /* PCG iterations on A                                   */
    int32_t n_outer;       /* refinement steps (mixed) or PCG restarts (FP64)       */
    double tau;            /* threshold used for Omega                              */
    double relres_after_local;  /* ||b - A x~|| / ||b|| after smoothing             */
    double relres_final;   /* ||b - A x|| / ||b|| of the returned x (FP64)         */
    double ms_construct, ms_local, ms_smooth, ms_global;  /* per-phase GPU time    */
} lcs_stats;

typedef struct lcs_ctx lcs_ctx;

/* Fill o with the defaults named above (eps 1e-10, Jacobi, FP64, 1 sweep). */
void lcs_default_options(lcs_options *o);

/* Create a context on the current HIP device.  Returns LCS_EHIP if no device. */
lcs_status lcs_create(lcs_ctx **ctx);
void lcs_destroy(lcs_ctx *ctx);

/* Bytes of a caller-owned device workspace (lcs_create_with_workspace) that
 * serves every single-system call on A with options o (NULL: the defaults of
 * lcs_default_options): a fixed head (device state, reduction partials) plus
 * every buffer the path may use at its largest.  The local domain is counted
 * at K = N, because Algorithms 2 and 3 may mark the whole grid, and general
 * sparse input counts its ELL copy and B at width 64.  About 240 B per row for the
 * nine-point stencil in mixed precision.  Host arithmetic only, no device
 * call.  Returns 0 if A or o is invalid (lcs_last_error() says why). */
size_t lcs_workspace_bytes(const lcs_matrix *A, const lcs_options *o);
/* The same for the batched calls on G systems of A's grid (1 <= G <= 65535). */
size_t lcs_workspace_bytes_batched(const lcs_matrix *A, int32_t G, const lcs_options *o);
/* Create a context on the current HIP device whose device state and buffers
 * all live in `workspace`: a caller-owned device buffer (for example a torch
 * uint8 tensor) of `bytes` bytes, 256-byte aligned, at least the fixed head.
 * Each call lays out the buffers it needs at its start and returns
 * LCS_EINVAL, before any work, if `bytes` is smaller than
 * lcs_workspace_bytes(A, o) of that call; it never allocates or frees device
 * memory and never synchronises the device (only its stream, where the call
 * needs a host decision).  The context's only allocations are made here:
 * small pinned host copies of the device state, and events.  The caller keeps
 * the buffer alive until lcs_destroy returns; the library never frees it.
 * LCS_EINVAL for a NULL or misaligned workspace or one below the head. */
lcs_status lcs_create_with_workspace(lcs_ctx **ctx, void *workspace, size_t bytes);
const char *lcs_last_error(void);

/* Global PCG from x (in: x^(0), out: solution) to eq. (rel-res-conv-criteria):
 * the baseline that Algorithm 1 is compared against (METHOD0's role). */
lcs_status lcs_solve_global(lcs_ctx *ctx, const lcs_matrix *A, const double *b, double *x,
                            const lcs_options *o, lcs_stats *st, void *stream);

/* Local domain (Algorithm 2 / Algorithm 3).  Writes idx[0..K) (device, capacity
 * N, ascending), *K (host) and, if mask != NULL, mask[N] (device uint8: 0 =
 * outside, 1 = marked by the threshold, m+1 = added by expansion round m).
 * e_max (0..250) is ignored in gradient mode.  st may be NULL. */
lcs_status lcs_build_local_domain(lcs_ctx *ctx, const lcs_matrix *A, const double *b,
                                  const double *x0, int32_t mode, int32_t thresh_kind,
                                  double theta, int32_t e_max, int32_t *idx, uint8_t *mask,
                                  int64_t *K, lcs_stats *st, void *stream);

/* lcs_build_local_domain for callers that cannot allocate device memory
 * (code under stream capture, tight serving loops, harnesses that forbid
 * hipMalloc): no context, and no allocation of any kind.  Its device state
 * and buffers live in one file-scope device array of 28 MiB that each GPU
 * holds from the library's load until the process ends; the call looks up
 * its address on the current device the first time.  Same arguments,
 * results (idx, *K, mask, stats) and errors as lcs_build_local_domain, bit
 * for bit, for the stencil kinds and N <= 2^21 cells (LCS_EINVAL for CSR
 * input or a larger N, before any work).  Every buffer is fully written
 * before it is read, so nothing needs clearing between calls.  All calls on
 * one GPU share the array: calls that overlap in time on one GPU (other
 * host threads, other streams) race and must be serialised by the caller.
 * Synchronises the stream. */
lcs_status lcs_build_local_domain_static(const lcs_matrix *A, const double *b, const double *x0,
                                         int32_t mode, int32_t thresh_kind, double theta,
                                         int32_t e_max, int32_t *idx, uint8_t *mask, int64_t *K,
                                         lcs_stats *st, void *stream);

/* Steps 3-7 of Algorithm 1 for a given Omega = idx[0..K) (device, ascending,
 * distinct): solve B d = r^(0)_Omega from d = 0 (the correction form of
 * eq. loc-equ), x <- x + d on Omega (eq. sol-assemble), then n_smooth
 * red-black Gauss-Seidel sweeps on A x = b.  x: in x^(0), out x~. */
lcs_status lcs_solve_local(lcs_ctx *ctx, const lcs_matrix *A, const double *b, double *x,
                           const int32_t *idx, int64_t K, const lcs_options *o,
                           lcs_stats *st, void *stream);

/* Algorithm 1: build Omega, solve locally, smooth, check, and finish with the
 * global PCG from x~ when needed.  x: in x^(0), out solution.  An x^(0) that
 * already meets the criterion ||b - A x^(0)||_2 <= eps ||b||_2 (eq.
 * rel-res-conv-criteria) is the solution and is returned unchanged: no local
 * solve, no smoothing, K = its_local = its_global = 0 (the global PCG does the
 * same with such an x^(0)). */
lcs_status lcs_solve_local_then_global(lcs_ctx *ctx, const lcs_matrix *A, const double *b,
                                       double *x, int32_t mode, int32_t thresh_kind,
                                       double theta, int32_t e_max, const lcs_options *o,
                                       lcs_stats *st, void *stream);

/* ---- pieces of the path, exported for parity tests and measurement ---- */

/* r = b - A x with the ascending-column FMA chain (score of Algorithm 3). */
lcs_status lcs_residual(lcs_ctx *ctx, const lcs_matrix *A, const double *b, const double *x,
                        double *r, void *stream);
/* g_i = sum_{j stored, j != i} |x_i - x_j| (eq. grad). */
lcs_status lcs_gradient(lcs_ctx *ctx, const lcs_matrix *A, const double *x, double *g,
                        void *stream);
/* y = A x; precision LCS_PREC_FP64 (x, y double) or LCS_PREC_MIXED (x, y float,
 * coefficients from A->coef32 or a cast).  reps launches back to back. */
lcs_status lcs_spmv(lcs_ctx *ctx, const lcs_matrix *A, const void *x, void *y,
                    int32_t precision, int32_t reps, void *stream);
/* Restricted B = A[idx, idx] in CSR (eq. BEFC): row_ptr int32[K+1],
 * col int32[nnz], val double[nnz] (device, capacity 9K; 16K for LCS_CSR).
 * *nnz (host). */
lcs_status lcs_gather_restricted(lcs_ctx *ctx, const lcs_matrix *A, const int32_t *idx,
                                 int64_t K, int32_t *row_ptr, int32_t *col, double *val,
                                 int64_t *nnz, void *stream);
/* n_sweeps red-black (9-point: four-colour) Gauss-Seidel sweeps on A x = b. */
lcs_status lcs_gs_sweeps(lcs_ctx *ctx, const lcs_matrix *A, const double *b, double *x,
                         int32_t n_sweeps, void *stream);
/* coef32 = (float) coef, n_arrays x N (device). */
lcs_status lcs_cast_coef(lcs_ctx *ctx, const lcs_matrix *A, float *coef32, void *stream);

/* ---- kernel timing for measurement ---- */
/* When on, every launch of the chosen kernel class goes through
 * hipExtLaunchKernelGGL with a start / stop event pair recorded by the
 * dispatch itself on the call's stream, so each interval is the kernel's
 * execution; the elapsed times are folded after each solve's final
 * synchronisation.  Setting a class (or LCS_TIME_NONE) resets the totals. */
enum {
    LCS_TIME_NONE = 0,
    LCS_TIME_LOCAL_AP = 1,        /* local PCG kernel that applies B: the whole
                                     iteration for Jacobi / none, q = B p for
                                     RB-SGS                                     */
    LCS_TIME_LOCAL_UPDATE = 2,    /* x, r, z update kernel of the local RB-SGS PCG */
    LCS_TIME_GLOBAL_AP = 3,       /* the same two classes for the global PCG    */
    LCS_TIME_GLOBAL_UPDATE = 4,
    LCS_TIME_SMOOTH = 5,          /* the Gauss-Seidel sweep kernels of Algorithm 1
                                     step 7 (and lcs_gs_sweeps)                 */
    LCS_TIME_SCORE = 6            /* the score kernel of the domain construction:
                                     r^(0) and its norms, or g (Algorithms 2, 3) */
};
lcs_status lcs_set_kernel_timing(lcs_ctx *ctx, int32_t what);
/* total milliseconds and number of timed launches since the last set */
lcs_status lcs_get_kernel_timing(lcs_ctx *ctx, double *ms_total, int64_t *launches);

/* ---- tiling of the stencil kernels ---- */
/* The grid-sized stencil kernels (nx a multiple of 4) walk the grid in one of
 * two ways: a flat walk (each thread takes strips in turn; neighbour rows are
 * re-read from cache), or row-marching tiles, where a wavefront owns 64
 * consecutive strips of one grid row (3-D: of one plane) and walks up
 * march_rows rows (3-D: planes), keeping the row (plane row) below in
 * registers, with non-temporal loads of the own-cell coefficient arrays and
 * non-temporal stores.  march_rows < 0 forces the flat walk,
 * 0 restores the automatic choice (marching once an FP64 pass streams more
 * than the 256 MB last-level cache, about 2048 tiles of at most 32 rows),
 * > 0 forces marching with that many rows; nontemporal 0 turns the
 * non-temporal hints of marching off, 1 or < 0 leaves them on.  Per-cell
 * results (residual, SpMV, scores, Gauss-Seidel) do not depend on these
 * settings; reductions may round differently. */
lcs_status lcs_set_tiling(lcs_ctx *ctx, int32_t march_rows, int32_t nontemporal);

/* Row order of the restricted system B under the red-black (multi-colour)
 * symmetric Gauss-Seidel preconditioner (precond = LCS_PC_RBSGS, 2..4
 * colours, symmetric operator).  on != 0 (the default): the local domain is
 * reordered colour by colour, ascending inside each colour, before B is
 * gathered, so that each half sweep of the preconditioner reads only the
 * rows of its own colour; on = 0: B keeps the ascending order of the domain
 * (Algorithm 1 step 3) and every half sweep walks all of B.  Each row keeps
 * its entries in ascending grid order, so every per-row result (z of each
 * half sweep, q = B p) is the same bit for bit either way; the reductions
 * (r.z, p.q) add the same terms in another order.  Returns LCS_EINVAL for a
 * NULL context. */
lcs_status lcs_set_colour_blocking(lcs_ctx *ctx, int32_t on);

/* Index form of the restricted system B (Algorithm 1 step 4) built by the
 * local solves.  on != 0 (the default): B's values sit in the stencil's
 * fixed slots and its columns are coded per row instead of a 32-bit index
 * per member, so that every product with B reads fewer bytes:
 *   - on the five- and nine-point stencils (LCS_STENCIL5_2D,
 *     LCS_STENCIL9_2D) with nx <= 32766, where B's rows keep the domain's
 *     ascending grid order: two 16-bit offsets to the rows below and above
 *     and the slots' presence bits (5 bytes), with only the upper slots'
 *     values stored (the lower couplings are read from the neighbours'
 *     mirrored slots, B being symmetric);
 *   - under RB-SGS with the rows blocked by colour (lcs_set_colour_blocking)
 *     on the five- and seven-point stencils (LCS_STENCIL7_3D), while half a
 *     row (2-D) or half a plane (3-D) holds at most 65535 cells: the row's
 *     position in the other colour's block, 16-bit distances to the members
 *     below and above, and the presence bits (9 or 13 bytes).
 * Otherwise, and with on = 0, as 32-bit indices.  B's members, their order
 * and every result are the same bit for bit either way.  Returns LCS_EINVAL
 * for a NULL context. */
lcs_status lcs_set_short_columns(lcs_ctx *ctx, int32_t on);

/* ---- batched solves: the G decoupled group systems of a source iteration ---- */
/* In each source iteration of the multi-group radiation diffusion equations
 * (Section 3.3, Algorithm 7) the G group equations are decoupled: G systems
 * A_g x_g = b_g on one grid and stencil kind.  These calls solve all G in one
 * launch, one workgroup per system, with the same results per system as the
 * single-system calls: lcs_solve_global_batched as lcs_solve_global, and
 * lcs_solve_local_then_global_batched as lcs_solve_local_then_global
 * (Algorithm 1, the same domain bit for bit, the same criterion).
 *   A->coef: device, G coefficient sets one after another, [G][n_arrays][N]
 *            (the layout of lcs_matrix per set); A->coef32 is ignored.
 *   b, x:    device, [G][N]; x in x^(0), out the solutions.
 *   st:      host array of G stats, or NULL; ms_* fields are 0 (one launch
 *            serves all systems: time the call).
 * The symmetric kinds run PCG; LCS_STENCIL9N_2D runs restarted GMRES(m)
 * (o->restart) in the local and the global solve, as the single-system
 * calls do, with a workspace of (m + 1) N doubles per system for the bases.
 * FP64 only (precision must be LCS_PREC_FP64), Jacobi or no preconditioner,
 * 1 <= G <= 65535, N <= 2^24 cells per system; otherwise LCS_EINVAL.  Every
 * system runs to completion; the call then returns the error of the first
 * system that failed (LCS_ENOCONV, LCS_EBREAKDOWN, LCS_ENONFINITE) with its
 * index in lcs_last_error(), or LCS_OK.  Synchronises the stream.  Intended
 * for small systems (about 10^3 - 10^5 cells each), where a solve through the
 * grid-wide kernels is bound by launch latency. */
lcs_status lcs_solve_global_batched(lcs_ctx *ctx, const lcs_matrix *A, int32_t G, const double *b,
                                    double *x, const lcs_options *o, lcs_stats *st, void *stream);
lcs_status lcs_solve_local_then_global_batched(lcs_ctx *ctx, const lcs_matrix *A, int32_t G,
                                               const double *b, double *x, int32_t mode,
                                               int32_t thresh_kind, double theta, int32_t e_max,
                                               const lcs_options *o, lcs_stats *st, void *stream);

/* ---- adjoint helpers (5- and 7-point log-conductivity operators) ---- */
/* coef = stencil of A = I*inv_dt + sum_f T_f (e_P-e_Q)(e_P-e_Q)^T with
 * T_f = 2 k_P k_Q / (k_P + k_Q), k = exp(logk); zero-flux outer faces. */
lcs_status lcs_assemble_logk(lcs_ctx *ctx, int32_t kind, int32_t nx, int32_t ny, int32_t nz,
                             double inv_dt, const double *logk, double *coef, void *stream);
/* grad_P = -sum_{faces (P,Q)} (dT_f/dlogk_P) (x_P - x_Q)(lambda_P - lambda_Q),
 * the derivative of lambda^T (b - A(logk) x) with respect to logk. */
lcs_status lcs_grad_logk(lcs_ctx *ctx, int32_t kind, int32_t nx, int32_t ny, int32_t nz,
                         const double *logk, const double *x, const double *lam,
                         double *grad, void *stream);

/* ---- the 2-D heat-conduction test problem (Section 3.1) ---- */
/* Picard system (eq. picard-equs) of dT/dt = div(k(T) grad T) with
 * k = T^power, T = t_left at x = 0, T = t_right at x = 1, zero flux at the
 * y faces: cell-centred finite volumes on nx x ny square cells of side
 * h = 1/nx (the unit square when ny = nx), scaled by h^2 (inv_dt = h^2/dt).  coef [3 x N] (C, E, N, the
 * 5-point layout of lcs_matrix) from k(t_lin); b [N] = t_old inv_dt plus the
 * Dirichlet terms.  Interior faces (k_P + k_Q) / 2; Dirichlet faces half a
 * cell away: 2 * (k_b + k_P) / 2, b += that * T_b.
 * Temperatures must be > 0 (k = exp(power log T)).  All arrays device. */
lcs_status lcs_assemble_heat(lcs_ctx *ctx, int32_t nx, int32_t ny, double inv_dt, double power,
                             double t_left, double t_right, const double *t_lin,
                             const double *t_old, double *coef, double *b, void *stream);
/* *out (host) = ||a - b||_2 over n entries (device arrays); synchronises the
 * stream.  The nonlinear (Picard) stopping test of the same section. */
lcs_status lcs_norm2_diff(lcs_ctx *ctx, const double *a, const double *b, int64_t n, double *out,
                          void *stream);

#ifdef __cplusplus
}
#endif
#endif /* LCS_H */
