/*
 * oracle.c -- plain, serial, FP64 reference of the local character-based
 * method (Ye, An, Xu: "A local character based method for solving linear
 * systems of radiation diffusion problems").
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may call this code;
 * only the tests, the smoke check and the CPU-baseline leg of the benchmark
 * load it.  It shares no code, header or table with the HIP library.
 *
 * Build: gcc -O2 -ffp-contract=off -fno-fast-math -shared -fPIC (no
 * contraction, so every product and sum below is rounded exactly as written;
 * fma() is used only where a fused step is stated).
 *
 * The same source built with -fopenmp (liboracle_omp.so) runs the loops
 * whose rows are independent on all host cores: residuals, products,
 * gradients, marking, an expansion round, Jacobi, the PCG vector updates
 * and one colour of a Gauss-Seidel sweep (rows of one colour never couple,
 * which the grid colourings guarantee).  Dot products, norms and the
 * compaction stay serial, so both builds return bit-identical results; the
 * parallel build exists to time the oracle on many cores, and the tests
 * check it against the serial one.
 *
 * Conventions (the readings of the paper are listed with each function):
 *   - A is CSR with ascending column indices per row; "a_ij != 0" of the
 *     paper is read as "a_ij is stored" (the structural pattern).
 *   - Every sum over a row runs over the stored entries in ascending column
 *     order.  Residuals use the chain acc = b_i; acc = fma(-a_ij, x_j, acc).
 *   - Dot products are serial sums in index order of rounded products.
 *   - All comparisons with thresholds are strict ">" as in the paper.
 *
 * Parity pins (see the CPU tests): the worked Example 1 (Section 2.3,
 * Table "extension process"), the five-point closed form of the gradient
 * (Section 2.2), dense direct solves, manufactured solutions, CG's finite
 * termination, brute-force set definitions, the adjoint's dense
 * derivative, and for the heat-conduction assembly the exactness of the
 * finite-volume scheme on linear profiles and its constant-coefficient limit.
 * No function here is "parity unpinned".
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* Host threads the row loops use: 1 in the serial build. */
int orc_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

#define ORC_OK 0
#define ORC_EINVAL 1
#define ORC_ENOCONV 4
#define ORC_EBREAKDOWN 5
#define ORC_ENOMEM 3

/* kinds of stencil input (symmetric storage, see the generator) */
#define ORC_K5 0
#define ORC_K9 1
#define ORC_K7 2
#define ORC_K9N 3 /* nine-point, full storage: array s = slot s of each row */

/* local-domain construction */
#define ORC_MODE_RESIDUAL 0 /* Section 2.3, Algorithm 3 */
#define ORC_MODE_GRADIENT 1 /* Section 2.2, Algorithm 2 */
#define ORC_TH_RELMAX 0     /* tau = theta * max_i s_i            */
#define ORC_TH_ABS 1        /* tau = theta                        */
#define ORC_TH_PAPER 2      /* tau = theta * ||b||_2 / sqrt(N), eq. (resi-local-domain-0) */

/* preconditioners */
#define ORC_PC_NONE 0
#define ORC_PC_JACOBI 1
#define ORC_PC_SGS 2 /* symmetric Gauss-Seidel in colour order */

/* ------------------------------------------------------------------ */
/* stencil -> CSR                                                      */
/* ------------------------------------------------------------------ */
/* Offsets of each stencil in ascending order of the neighbour's index. */
static const int OFF5[5][3] = {{0, -1, 0}, {-1, 0, 0}, {0, 0, 0}, {1, 0, 0}, {0, 1, 0}};
static const int OFF9[9][3] = {{-1, -1, 0}, {0, -1, 0}, {1, -1, 0}, {-1, 0, 0}, {0, 0, 0},
                               {1, 0, 0},   {-1, 1, 0}, {0, 1, 0},  {1, 1, 0}};
static const int OFF7[7][3] = {{0, 0, -1}, {0, -1, 0}, {-1, 0, 0}, {0, 0, 0},
                               {1, 0, 0},  {0, 1, 0},  {0, 0, 1}};

static int stencil_offsets(int kind, const int (**off)[3]) {
    switch (kind) {
    case ORC_K5: *off = OFF5; return 5;
    case ORC_K9: *off = OFF9; return 9;
    case ORC_K9N: *off = OFF9; return 9;
    case ORC_K7: *off = OFF7; return 7;
    default: return 0;
    }
}

/* Value a(P, P+d) from symmetric storage.  coef rows:
 *   5pt: C,E,N   9pt: C,E,N,NE,NW   7pt: C,E,N,U
 * A backward coupling is the forward coupling stored at the neighbour. */
static double stencil_value(int kind, const double *coef, int64_t n, int64_t p,
                            int dx, int dy, int dz, int64_t sx, int64_t sy) {
    int64_t q = p + dx + dy * sx + dz * sy;
    if (kind == ORC_K9N) return coef[(int64_t)((dy + 1) * 3 + (dx + 1)) * n + p];
    if (dx == 0 && dy == 0 && dz == 0) return coef[p];
    const double *E = coef + n, *N = coef + 2 * n;
    if (dz == 0 && dy == 0) return dx > 0 ? E[p] : E[q];
    if (dz == 0 && dx == 0) return dy > 0 ? N[p] : N[q];
    if (kind == ORC_K9) {
        const double *NE = coef + 3 * n, *NW = coef + 4 * n;
        if (dx == dy) return dy > 0 ? NE[p] : NE[q];
        return dy > 0 ? NW[p] : NW[q]; /* (-1,+1) from p, or (+1,-1) = NW of q */
    }
    if (kind == ORC_K7) {
        const double *U = coef + 3 * n;
        return dz > 0 ? U[p] : U[q];
    }
    return 0.0;
}

int64_t orc_stencil_nnz(int kind, int nx, int ny, int nz) {
    const int (*off)[3];
    int m = stencil_offsets(kind, &off);
    int64_t nnz = 0;
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x)
                for (int s = 0; s < m; ++s) {
                    int X = x + off[s][0], Y = y + off[s][1], Z = z + off[s][2];
                    if (X >= 0 && X < nx && Y >= 0 && Y < ny && Z >= 0 && Z < nz) ++nnz;
                }
    return nnz;
}

/* All in-grid neighbours of the stencil are stored (the structural pattern),
 * columns ascending. */
int orc_csr_from_stencil(int kind, int nx, int ny, int nz, const double *coef,
                         int64_t *rp, int32_t *col, double *val) {
    const int (*off)[3];
    int m = stencil_offsets(kind, &off);
    if (!m) return ORC_EINVAL;
    int64_t n = (int64_t)nx * ny * nz, sx = nx, sy = (int64_t)nx * ny, k = 0;
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                int64_t p = x + sx * y + sy * z;
                rp[p] = k;
                for (int s = 0; s < m; ++s) {
                    int X = x + off[s][0], Y = y + off[s][1], Z = z + off[s][2];
                    if (X < 0 || X >= nx || Y < 0 || Y >= ny || Z < 0 || Z >= nz) continue;
                    col[k] = (int32_t)(p + off[s][0] + off[s][1] * sx + off[s][2] * sy);
                    val[k] = stencil_value(kind, coef, n, p, off[s][0], off[s][1], off[s][2], sx, sy);
                    ++k;
                }
            }
    rp[n] = k;
    return ORC_OK;
}

/* Colour of each cell for red-black (2 colours: parity of x+y+z) or, for the
 * nine-point stencil, 4 colours (parity of x) + 2*(parity of y). */
int orc_grid_colours(int kind, int nx, int ny, int nz, int8_t *colour) {
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                int64_t p = x + (int64_t)nx * y + (int64_t)nx * ny * z;
                colour[p] = (int8_t)(kind == ORC_K9 || kind == ORC_K9N ? (x & 1) + 2 * (y & 1)
                                                                      : (x + y + z) & 1);
            }
    return kind == ORC_K9 || kind == ORC_K9N ? 4 : 2;
}

/* ------------------------------------------------------------------ */
/* elementary operations                                               */
/* ------------------------------------------------------------------ */
/* r = b - A x.  Component form of the residual (Section 2.3.1). */
void orc_residual(int64_t n, const int64_t *rp, const int32_t *col, const double *val,
                  const double *b, const double *x, double *r) {
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double acc = b[i];
        for (int64_t k = rp[i]; k < rp[i + 1]; ++k) acc = fma(-val[k], x[col[k]], acc);
        r[i] = acc;
    }
}

/* y = A x */
void orc_spmv(int64_t n, const int64_t *rp, const int32_t *col, const double *val,
              const double *x, double *y) {
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double acc = 0.0;
        for (int64_t k = rp[i]; k < rp[i + 1]; ++k) acc = fma(val[k], x[col[k]], acc);
        y[i] = acc;
    }
}

double orc_dot(int64_t n, const double *a, const double *b) {
    double s = 0.0;
    for (int64_t i = 0; i < n; ++i) s += a[i] * b[i];
    return s;
}

double orc_norm2(int64_t n, const double *a) { return sqrt(orc_dot(n, a, a)); }

/* Gradient mimic g_i = sum over stored j of |x_i - x_j|, eq. (grad),
 * Section 2.2.  The j = i term is |0| and is left out (it adds +0). */
void orc_gradient(int64_t n, const int64_t *rp, const int32_t *col, const double *x, double *g) {
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double s = 0.0;
        for (int64_t k = rp[i]; k < rp[i + 1]; ++k) {
            int64_t j = col[k];
            if (j != i) s += fabs(x[i] - x[j]);
        }
        g[i] = s;
    }
}

/* ------------------------------------------------------------------ */
/* local-domain construction (Algorithms 2 and 3)                      */
/* ------------------------------------------------------------------ */
/*
 * mask[i] (out) = 0 if i is not in the local domain, 1 if it was marked by
 * the threshold, m+1 if expansion round m added it.
 * score (out, n)  = r^(0) (residual mode) or g (gradient mode).
 * idx (out, cap n) = ascending indices of the local domain; *K its size.
 * *rounds (out)   = expansion rounds that added points.
 * *tau (out)      = the threshold used.
 *
 * Residual mode (Section 2.3, Algorithm 3):
 *   r^(0) = b - A x^(0); Omega = {i : |r_i| > tau};
 *   for m = 1..e_max: candidates are j not in Omega with a stored a_jl,
 *   l in Omega; s_j = |r_j| + sum_{l in Omega, ascending} |a_jl x_l|
 *   (eq. extend-local-condition); j joins if s_j > tau.  Omega is the set at
 *   the start of the round (additions take effect after the sweep); the loop
 *   stops at the first round that adds nothing.
 * Gradient mode (Section 2.2, Algorithm 2): g from eq. (grad);
 *   Omega = {i : g_i > tau}.  There is no expansion in Algorithm 2.
 * Thresholds: RELMAX tau = theta * max_i |s_i| (alpha * g_max of Algorithm 2;
 *   a max-norm-relative residual threshold), ABS tau = theta, PAPER
 *   tau = theta * ||b||_2 / sqrt(N) with theta = epsilon (eq.
 *   resi-local-domain-0).
 */
int orc_build_local_domain(int64_t n, const int64_t *rp, const int32_t *col, const double *val,
                           const double *b, const double *x0, int mode, int thresh_kind,
                           double theta, int e_max, uint8_t *mask, int32_t *idx, int64_t *K,
                           int *rounds, double *tau_out, double *score) {
    if (n <= 0) { *K = 0; *rounds = 0; *tau_out = 0.0; return ORC_OK; }
    if (e_max < 0 || e_max > 250) return ORC_EINVAL;
    if (mode == ORC_MODE_RESIDUAL) orc_residual(n, rp, col, val, b, x0, score);
    else if (mode == ORC_MODE_GRADIENT) orc_gradient(n, rp, col, x0, score);
    else return ORC_EINVAL;

    double tau;
    if (thresh_kind == ORC_TH_RELMAX) {
        double m = 0.0;
#pragma omp parallel for schedule(static) reduction(max : m)
        for (int64_t i = 0; i < n; ++i) {
            double s = fabs(score[i]);
            if (s > m) m = s;
        }
        tau = theta * m;
    } else if (thresh_kind == ORC_TH_ABS) {
        tau = theta;
    } else if (thresh_kind == ORC_TH_PAPER && mode == ORC_MODE_RESIDUAL) {
        tau = theta * orc_norm2(n, b) / sqrt((double)n);
    } else {
        return ORC_EINVAL;
    }
    *tau_out = tau;

#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) mask[i] = fabs(score[i]) > tau ? 1 : 0;

    int grown = 0;
    if (mode == ORC_MODE_RESIDUAL) {
        uint8_t *in_start = (uint8_t *)malloc((size_t)n);
        if (!in_start) return ORC_ENOMEM;
        for (int m = 1; m <= e_max; ++m) {
            for (int64_t i = 0; i < n; ++i) in_start[i] = mask[i] != 0;
            int64_t added = 0;
#pragma omp parallel for schedule(static) reduction(+ : added)
            for (int64_t j = 0; j < n; ++j) {
                if (in_start[j]) continue;
                int neighbour = 0;
                double s = fabs(score[j]);
                for (int64_t k = rp[j]; k < rp[j + 1]; ++k) {
                    int64_t l = col[k];
                    if (in_start[l]) {
                        neighbour = 1;
                        s += fabs(val[k] * x0[l]);
                    }
                }
                if (neighbour && s > tau) {
                    mask[j] = (uint8_t)(m + 1);
                    ++added;
                }
            }
            if (added == 0) break;
            ++grown;
        }
        free(in_start);
    }
    *rounds = grown;

    int64_t k = 0;
    for (int64_t i = 0; i < n; ++i)
        if (mask[i]) idx[k++] = (int32_t)i;
    *K = k;
    return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* restricted subsystem (eq. BEFC, eq. loc-equ)                        */
/* ------------------------------------------------------------------ */
/* inv[i] = position of i in idx, or -1.  B = A[idx, idx] with columns
 * renumbered through inv (inv is monotone on idx, so order is kept). */
int64_t orc_restricted_nnz(int64_t n, const int64_t *rp, const int32_t *col, const int32_t *idx,
                           int64_t K, int32_t *inv) {
    for (int64_t i = 0; i < n; ++i) inv[i] = -1;
    for (int64_t k = 0; k < K; ++k) inv[idx[k]] = (int32_t)k;
    int64_t nnz = 0;
    for (int64_t k = 0; k < K; ++k)
        for (int64_t e = rp[idx[k]]; e < rp[idx[k] + 1]; ++e)
            if (inv[col[e]] >= 0) ++nnz;
    return nnz;
}

void orc_restricted(const int64_t *rp, const int32_t *col, const double *val, const int32_t *idx,
                    int64_t K, const int32_t *inv, int64_t *brp, int32_t *bcol, double *bval) {
    int64_t t = 0;
    for (int64_t k = 0; k < K; ++k) {
        brp[k] = t;
        for (int64_t e = rp[idx[k]]; e < rp[idx[k] + 1]; ++e) {
            int32_t c = inv[col[e]];
            if (c >= 0) {
                bcol[t] = c;
                bval[t] = val[e];
                ++t;
            }
        }
    }
    brp[K] = t;
}

/* ------------------------------------------------------------------ */
/* preconditioned conjugate gradients                                  */
/* ------------------------------------------------------------------ */
static double diag_of(const int64_t *rp, const int32_t *col, const double *val, int64_t i) {
    for (int64_t k = rp[i]; k < rp[i + 1]; ++k)
        if (col[k] == i) return val[k];
    return 0.0;
}

/* One Gauss-Seidel update of every row of colour c:
 * x_i = (rhs_i - sum_{j != i, ascending} a_ij x_j) / a_ii. */
static void gs_colour(int64_t n, const int64_t *rp, const int32_t *col, const double *val,
                      const double *rhs, double *x, const int8_t *colour, int c) {
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        if (colour[i] != c) continue;
        double acc = rhs[i], d = 0.0;
        for (int64_t k = rp[i]; k < rp[i + 1]; ++k) {
            if (col[k] == i) { d = val[k]; continue; }
            acc = fma(-val[k], x[col[k]], acc);
        }
        x[i] = acc / d;
    }
}

/* z = M^-1 r */
static void apply_precond(int64_t n, const int64_t *rp, const int32_t *col, const double *val,
                          int pc, const double *diag, const int8_t *colour, int ncol,
                          const double *r, double *z) {
    if (pc == ORC_PC_JACOBI) {
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < n; ++i) z[i] = r[i] / diag[i];
    } else if (pc == ORC_PC_SGS) {
        /* symmetric GS from z = 0: colours forward then backward */
        for (int64_t i = 0; i < n; ++i) z[i] = 0.0;
        for (int c = 0; c < ncol; ++c) gs_colour(n, rp, col, val, r, z, colour, c);
        for (int c = ncol - 1; c >= 0; --c) gs_colour(n, rp, col, val, r, z, colour, c);
    } else {
        for (int64_t i = 0; i < n; ++i) z[i] = r[i];
    }
}

/*
 * PCG for SPD A from the initial x (in/out), until the recursive residual
 * satisfies ||r||_2 <= tol_abs (the criterion eq. rel-res-conv-criteria with
 * tol_abs = epsilon ||b||_2), or max_iter iterations.
 * Standard recurrences (Hestenes-Stiefel with a preconditioner):
 *   r = b - A x; z = M^-1 r; p = z; rz = r.z
 *   repeat: q = A p; alpha = rz / p.q; x += alpha p; r -= alpha q;
 *           stop if ||r|| <= tol; z = M^-1 r; beta = r.z_new / rz; p = z + beta p
 * Returns ORC_OK, ORC_ENOCONV (max_iter reached) or ORC_EBREAKDOWN (p.q <= 0).
 * *iters = iterations done, *res = recursive ||r||_2 at exit.
 */
int orc_pcg(int64_t n, const int64_t *rp, const int32_t *col, const double *val, const double *b,
            double *x, int pc, const int8_t *colour, int ncol, double tol_abs, int max_iter,
            int *iters, double *res) {
    *iters = 0;
    if (n == 0) { *res = 0.0; return ORC_OK; }
    double *r = malloc(sizeof(double) * n), *z = malloc(sizeof(double) * n);
    double *p = malloc(sizeof(double) * n), *q = malloc(sizeof(double) * n);
    double *diag = malloc(sizeof(double) * n);
    if (!r || !z || !p || !q || !diag) { free(r); free(z); free(p); free(q); free(diag); return ORC_ENOMEM; }
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) diag[i] = diag_of(rp, col, val, i);
    orc_residual(n, rp, col, val, b, x, r);
    double rr = orc_dot(n, r, r);
    int status = ORC_ENOCONV, it = 0;
    if (sqrt(rr) <= tol_abs) {
        status = ORC_OK;
    } else {
        apply_precond(n, rp, col, val, pc, diag, colour, ncol, r, z);
        memcpy(p, z, sizeof(double) * n);
        double rz = orc_dot(n, r, z);
        while (it < max_iter) {
            orc_spmv(n, rp, col, val, p, q);
            double pq = orc_dot(n, p, q);
            if (!(pq > 0.0)) { status = ORC_EBREAKDOWN; break; }
            double alpha = rz / pq;
#pragma omp parallel for schedule(static)
            for (int64_t i = 0; i < n; ++i) {
                x[i] = fma(alpha, p[i], x[i]);
                r[i] = fma(-alpha, q[i], r[i]);
            }
            ++it;
            rr = orc_dot(n, r, r);
            if (sqrt(rr) <= tol_abs) { status = ORC_OK; break; }
            apply_precond(n, rp, col, val, pc, diag, colour, ncol, r, z);
            double rz_new = orc_dot(n, r, z);
            double beta = rz_new / rz;
            rz = rz_new;
#pragma omp parallel for schedule(static)
            for (int64_t i = 0; i < n; ++i) p[i] = fma(beta, p[i], z[i]);
        }
    }
    *iters = it;
    *res = sqrt(rr);
    free(r); free(z); free(p); free(q); free(diag);
    return status;
}

/* n_sweeps Gauss-Seidel sweeps on A x = b, colours 0..ncol-1 in turn
 * (the smoothing step of Algorithm 1). */
void orc_gs_sweeps(int64_t n, const int64_t *rp, const int32_t *col, const double *val,
                   const double *b, double *x, const int8_t *colour, int ncol, int n_sweeps) {
    for (int s = 0; s < n_sweeps; ++s)
        for (int c = 0; c < ncol; ++c) gs_colour(n, rp, col, val, b, x, colour, c);
}

/*
 * Restarted GMRES(m) for a general (non-symmetric) A, the Krylov method of
 * the paper's experiments (Section 3), right-preconditioned:
 * A M^-1 u = r0, x = x0 + M^-1 u, with M = diag(A) (ORC_PC_JACOBI) or I.
 * Each cycle: r = b - A x, beta = ||r||; stop if beta <= tol_abs;
 * v_0 = r / beta, g = beta e_1; for j = 0..m-1: w = A M^-1 v_j; modified
 * Gram-Schmidt h_ij = v_i . w, w -= h_ij v_i (i = 0..j); h_{j+1,j} = ||w||;
 * the Givens rotations of columns 0..j-1 are applied to column j, a new one
 * (c, s) = (h_jj, h_{j+1,j}) / sqrt(h_jj^2 + h_{j+1,j}^2) zeroes h_{j+1,j}
 * and g_{j+1} = -s g_j, g_j = c g_j; |g_{j+1}| is ||b - A x_j||; stop the
 * cycle when it is <= tol_abs, when h_{j+1,j} = 0, or after m steps;
 * v_{j+1} = w / h_{j+1,j}.  Then H y = g by back substitution over the k
 * columns, and x += M^-1 (sum_i y_i v_i).  Cycles repeat until the estimate
 * meets tol_abs or max_iter steps were taken.
 * Returns ORC_OK, ORC_ENOCONV or ORC_EBREAKDOWN (a zero column: singular
 * A M^-1); *iters = Arnoldi steps, *res = the last residual estimate.
 */
int orc_gmres(int64_t n, const int64_t *rp, const int32_t *col, const double *val, const double *b,
              double *x, int pc, int m, double tol_abs, int max_iter, int *iters, double *res) {
    *iters = 0;
    *res = 0.0;
    if (n == 0) return ORC_OK;
    if (m < 1) m = 1;
    double *V = malloc(sizeof(double) * (size_t)(m + 1) * n);
    double *w = malloc(sizeof(double) * n), *z = malloc(sizeof(double) * n);
    double *diag = malloc(sizeof(double) * n);
    double *H = calloc((size_t)(m + 1) * m, sizeof(double));
    double *cs = malloc(sizeof(double) * m), *sn = malloc(sizeof(double) * m);
    double *g = malloc(sizeof(double) * (m + 1)), *y = malloc(sizeof(double) * m);
    if (!V || !w || !z || !diag || !H || !cs || !sn || !g || !y) {
        free(V); free(w); free(z); free(diag); free(H); free(cs); free(sn); free(g); free(y);
        return ORC_ENOMEM;
    }
    for (int64_t i = 0; i < n; ++i) diag[i] = diag_of(rp, col, val, i);
#define HH(i, j) H[(size_t)(j) * (m + 1) + (i)]
    int status = ORC_ENOCONV, it = 0;
    for (;;) {
        orc_residual(n, rp, col, val, b, x, w);
        double beta = orc_norm2(n, w);
        *res = beta;
        if (beta <= tol_abs) { status = ORC_OK; break; }
        if (it >= max_iter) break;
        for (int64_t i = 0; i < n; ++i) V[i] = w[i] / beta;
        for (int q = 0; q <= m; ++q) g[q] = 0.0;
        g[0] = beta;
        int k = 0, stop = 0;
        for (int j = 0; j < m && it < max_iter; ++j) {
            const double *vj = V + (size_t)j * n;
            for (int64_t i = 0; i < n; ++i) z[i] = pc == ORC_PC_JACOBI ? vj[i] / diag[i] : vj[i];
            orc_spmv(n, rp, col, val, z, w);
            for (int i = 0; i <= j; ++i) {
                const double *vi = V + (size_t)i * n;
                double h = orc_dot(n, vi, w);
                HH(i, j) = h;
                for (int64_t l = 0; l < n; ++l) w[l] = fma(-h, vi[l], w[l]);
            }
            double hn = orc_norm2(n, w);
            HH(j + 1, j) = hn;
            for (int i = 0; i < j; ++i) {
                double t = cs[i] * HH(i, j) + sn[i] * HH(i + 1, j);
                HH(i + 1, j) = -sn[i] * HH(i, j) + cs[i] * HH(i + 1, j);
                HH(i, j) = t;
            }
            double a = HH(j, j), bb = HH(j + 1, j);
            double den = sqrt(a * a + bb * bb);
            ++it;
            if (!(den > 0.0)) { status = ORC_EBREAKDOWN; stop = 2; k = j; break; }
            cs[j] = a / den;
            sn[j] = bb / den;
            HH(j, j) = den;
            HH(j + 1, j) = 0.0;
            g[j + 1] = -sn[j] * g[j];
            g[j] = cs[j] * g[j];
            *res = fabs(g[j + 1]);
            k = j + 1;
            if (*res <= tol_abs || hn == 0.0) { stop = 1; break; }
            double *vn = V + (size_t)(j + 1) * n;
            for (int64_t l = 0; l < n; ++l) vn[l] = w[l] / hn;
        }
        for (int i = k - 1; i >= 0; --i) {
            double acc = g[i];
            for (int l = i + 1; l < k; ++l) acc -= HH(i, l) * y[l];
            y[i] = acc / HH(i, i);
        }
        for (int64_t l = 0; l < n; ++l) {
            double u = 0.0;
            for (int q = 0; q < k; ++q) u = fma(y[q], V[(size_t)q * n + l], u);
            if (pc == ORC_PC_JACOBI) u = u / diag[l];
            x[l] += u;
        }
        if (stop == 2) break;
        if (stop == 1) { status = ORC_OK; break; }
        if (it >= max_iter) break;
    }
#undef HH
    *iters = it;
    free(V); free(w); free(z); free(diag); free(H); free(cs); free(sn); free(g); free(y);
    return status;
}

/* ------------------------------------------------------------------ */
/* Algorithm 1                                                         */
/* ------------------------------------------------------------------ */
typedef struct {
    double eps;       /* global criterion ||b - Ax|| <= eps ||b|| */
    double tol_local; /* local criterion ||rhs_B - B d|| <= tol_local ||b|| */
    int max_iter;
    int pc;           /* ORC_PC_* */
    int n_smooth;     /* GS sweeps applied to x~ */
    int max_restart;  /* global restarts after a failed true-residual check */
    int krylov;       /* ORC_KRYLOV_CG (SPD A) or ORC_KRYLOV_GMRES (any A) */
    int gmres_m;      /* GMRES restart length */
} orc_opts;

#define ORC_KRYLOV_CG 0
#define ORC_KRYLOV_GMRES 1

/* The Krylov solve of Algorithm 1's local and global steps: PCG for SPD A,
 * GMRES(m) otherwise (same arguments). */
static int orc_krylov(int64_t n, const int64_t *rp, const int32_t *col, const double *val,
                      const double *b, double *x, const orc_opts *o, const int8_t *colour,
                      int ncol, double tol_abs, int max_iter, int *iters, double *res) {
    if (o->krylov == ORC_KRYLOV_GMRES)
        return orc_gmres(n, rp, col, val, b, x, o->pc, o->gmres_m, tol_abs, max_iter, iters, res);
    return orc_pcg(n, rp, col, val, b, x, o->pc, colour, ncol, tol_abs, max_iter, iters, res);
}

typedef struct {
    int64_t K;
    int its_local, its_global, restarts, status_local;
    double relres_after_local, relres_final;
} orc_stats;

/* Global solve from x (in/out): run PCG, verify the true residual, restart
 * from the current x while it fails (at most max_restart times). */
int orc_solve_global(int64_t n, const int64_t *rp, const int32_t *col, const double *val,
                     const double *b, double *x, const int8_t *colour, int ncol,
                     const orc_opts *o, orc_stats *st) {
    double nb = orc_norm2(n, b), tol = o->eps * nb;
    double *r = malloc(sizeof(double) * (n > 0 ? n : 1));
    if (!r) return ORC_ENOMEM;
    int status = ORC_OK, total = 0;
    st->restarts = 0;
    for (int attempt = 0;; ++attempt) {
        int it; double res;
        status = orc_krylov(n, rp, col, val, b, x, o, colour, ncol, tol, o->max_iter - total, &it, &res);
        total += it;
        orc_residual(n, rp, col, val, b, x, r);
        double tr = orc_norm2(n, r);
        st->relres_final = nb > 0 ? tr / nb : tr;
        if (status != ORC_OK) break;
        if (tr <= tol) break;
        if (attempt >= o->max_restart || total >= o->max_iter) { status = ORC_ENOCONV; break; }
        st->restarts++;
    }
    st->its_global = total;
    free(r);
    return status;
}

/* Steps 3-7 of Algorithm 1 for a given local domain idx[0..K):
 * B d = r^(0)_Omega from d = 0 (the correction form of eq. loc-equ:
 * b_B - E x_C^(0) - B x_B^(0) = r^(0)_B), x~ = x^(0) with x~_Omega += d
 * (eq. sol-assemble), then n_smooth GS sweeps on the global system. */
int orc_solve_local(int64_t n, const int64_t *rp, const int32_t *col, const double *val,
                    const double *b, double *x, const int32_t *idx, int64_t K,
                    const int8_t *colour, int ncol, const orc_opts *o, orc_stats *st) {
    st->K = K;
    st->its_local = 0;
    st->status_local = ORC_OK;
    double nb = orc_norm2(n, b);
    if (K > 0) {
        int32_t *inv = malloc(sizeof(int32_t) * n);
        double *r = malloc(sizeof(double) * n);
        if (!inv || !r) { free(inv); free(r); return ORC_ENOMEM; }
        orc_residual(n, rp, col, val, b, x, r);
        int64_t bnnz = orc_restricted_nnz(n, rp, col, idx, K, inv);
        int64_t *brp = malloc(sizeof(int64_t) * (K + 1));
        int32_t *bcol = malloc(sizeof(int32_t) * (bnnz > 0 ? bnnz : 1));
        double *bval = malloc(sizeof(double) * (bnnz > 0 ? bnnz : 1));
        double *rhs = malloc(sizeof(double) * K), *d = calloc((size_t)K, sizeof(double));
        int8_t *bcolour = malloc((size_t)K);
        if (!brp || !bcol || !bval || !rhs || !d || !bcolour) return ORC_ENOMEM;
        orc_restricted(rp, col, val, idx, K, inv, brp, bcol, bval);
        for (int64_t k = 0; k < K; ++k) {
            rhs[k] = r[idx[k]];
            bcolour[k] = colour ? colour[idx[k]] : 0;
        }
        int it; double res;
        st->status_local = orc_krylov(K, brp, bcol, bval, rhs, d, o, bcolour, ncol,
                                      o->tol_local * nb, o->max_iter, &it, &res);
        st->its_local = it;
        for (int64_t k = 0; k < K; ++k) x[idx[k]] += d[k];
        free(inv); free(r); free(brp); free(bcol); free(bval); free(rhs); free(d); free(bcolour);
    }
    if (o->n_smooth > 0 && colour)
        orc_gs_sweeps(n, rp, col, val, b, x, colour, ncol, o->n_smooth);
    double *r2 = malloc(sizeof(double) * (n > 0 ? n : 1));
    orc_residual(n, rp, col, val, b, x, r2);
    st->relres_after_local = nb > 0 ? orc_norm2(n, r2) / nb : orc_norm2(n, r2);
    free(r2);
    return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* adjoint helpers for the five/seven-point log-conductivity operator  */
/* ------------------------------------------------------------------ */
/* A = I/dt + sum_f T_f (e_P - e_Q)(e_P - e_Q)^T, T_f = 2 k_P k_Q/(k_P + k_Q),
 * k = exp(l).  Writes symmetric stencil rows C,E,N(,U). */
int orc_assemble_logk(int kind, int nx, int ny, int nz, double inv_dt, const double *logk,
                      double *coef) {
    if (kind != ORC_K5 && kind != ORC_K7) return ORC_EINVAL;
    int64_t n = (int64_t)nx * ny * nz, sx = nx, sy = (int64_t)nx * ny;
    int nd = kind == ORC_K5 ? 2 : 3;
    for (int64_t i = 0; i < n; ++i) coef[i] = inv_dt;
    for (int a = 1; a <= nd; ++a)
        for (int64_t i = 0; i < n; ++i) coef[a * n + i] = 0.0;
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                int64_t p = x + sx * y + sy * z;
                int has[3] = {x + 1 < nx, y + 1 < ny, z + 1 < nz};
                int64_t step[3] = {1, sx, sy};
                for (int a = 0; a < nd; ++a) {
                    if (!has[a]) continue;
                    int64_t q = p + step[a];
                    double kp = exp(logk[p]), kq = exp(logk[q]);
                    double t = 2.0 * kp * kq / (kp + kq);
                    coef[(a + 1) * n + p] = -t;
                    coef[p] += t;
                    coef[q] += t;
                }
            }
    return ORC_OK;
}

/* dL/dl_P = -lambda^T (dA/dl_P) x = -sum_{faces f=(P,Q)} (dT_f/dl_P)(x_P - x_Q)(lambda_P - lambda_Q)
 * with dT_f/dl_P = T_f k_Q / (k_P + k_Q).  Faces in ascending neighbour order. */
int orc_grad_logk(int kind, int nx, int ny, int nz, const double *logk, const double *xs,
                  const double *lam, double *grad) {
    if (kind != ORC_K5 && kind != ORC_K7) return ORC_EINVAL;
    int64_t sx = nx, sy = (int64_t)nx * ny;
    const int (*off)[3];
    int m = stencil_offsets(kind, &off);
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                int64_t p = x + sx * y + sy * z;
                double kp = exp(logk[p]), s = 0.0;
                for (int e = 0; e < m; ++e) {
                    int X = x + off[e][0], Y = y + off[e][1], Z = z + off[e][2];
                    if (off[e][0] == 0 && off[e][1] == 0 && off[e][2] == 0) continue;
                    if (X < 0 || X >= nx || Y < 0 || Y >= ny || Z < 0 || Z >= nz) continue;
                    int64_t q = X + sx * Y + sy * Z;
                    double kq = exp(logk[q]);
                    double t = 2.0 * kp * kq / (kp + kq);
                    double dt = t * kq / (kp + kq);
                    s += dt * (xs[p] - xs[q]) * (lam[p] - lam[q]);
                }
                grad[p] = -s;
            }
    return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* 2-D nonlinear heat conduction test problem (Section 3.1)            */
/* ------------------------------------------------------------------ */
/* Picard system of dT/dt = div(k(T) grad T) on the unit square, k = T^power,
 * T = tl at x = 0 and T = tr at x = 1, zero flux at y = 0 and y = 1, backward
 * Euler (eq. picard-equs).  Reading (the paper says only "five-point finite
 * difference"): cell-centred finite volumes, nx x ny cells of width
 * h = 1/nx, the equation multiplied by h^2, so
 *   A = I h^2/dt + sum_faces t_f (e_P - e_Q)(e_P - e_Q)^T + Dirichlet faces,
 *   t_f = (k_P + k_Q) / 2, the arithmetic mean of the two cells' k, on
 *         interior faces (the harmonic mean would shut the face between a
 *         hot cell and a cold one, k(1e-4) = 1e-14, and freeze the front
 *         that the paper's local domains follow across the time steps);
 *   t_b = 2 * (k_b + k_P) / 2 on an x boundary face (half a cell to the
 *         boundary value), k_b = k(tl) or k(tr), with b gaining t_b T_b;
 *   b = T_old h^2/dt + boundary terms.
 * k(T) = exp(power * log(T)).  Diagonal sums in the order inv_dt, west,
 * east, south, north.  coef = [C, E, N] (symmetric storage). */
static double orc_kpow(double t, double power) { return exp(power * log(t)); }
static double orc_mean(double a, double b) { return 0.5 * (a + b); }

int orc_heat_assemble(int nx, int ny, double inv_dt, double power, double tl, double tr,
                      const double *tlin, const double *told, double *coef, double *b) {
    if (nx < 1 || ny < 1) return ORC_EINVAL;
    int64_t n = (int64_t)nx * ny;
    double kl = orc_kpow(tl, power), kr = orc_kpow(tr, power);
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            int64_t p = x + (int64_t)nx * y;
            double kp = orc_kpow(tlin[p], power);
            double tw = x > 0 ? orc_mean(orc_kpow(tlin[p - 1], power), kp) : 2.0 * orc_mean(kl, kp);
            double te = x < nx - 1 ? orc_mean(kp, orc_kpow(tlin[p + 1], power)) : 2.0 * orc_mean(kp, kr);
            double ts = y > 0 ? orc_mean(orc_kpow(tlin[p - nx], power), kp) : 0.0;
            double tn = y < ny - 1 ? orc_mean(kp, orc_kpow(tlin[p + nx], power)) : 0.0;
            double d = inv_dt;
            d += tw;
            d += te;
            d += ts;
            d += tn;
            coef[p] = d;
            coef[n + p] = x < nx - 1 ? -te : 0.0;
            coef[2 * n + p] = y < ny - 1 ? -tn : 0.0;
            double r = told[p] * inv_dt;
            if (x == 0) r += tw * tl;
            if (x == nx - 1) r += te * tr;
            b[p] = r;
        }
    return ORC_OK;
}
