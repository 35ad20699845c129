// Batched solves: G independent systems on one grid, one workgroup each.
//
// In a source iteration of the multi-group radiation diffusion equations the
// G group equations are decoupled (Algorithm 7): G systems A_g x_g = b_g of
// the same grid and stencil, each small (thousands of cells).  A solve of one
// such system through the grid-wide kernels is a chain of a few hundred
// launches, each far too small to fill the chip, so its time is launch and
// synchronisation latency.  Here one workgroup of 1024 threads runs the whole
// of Algorithm 1 for one system (scores, threshold, expansion rounds,
// compaction, local PCG on Omega, assembly, Gauss-Seidel sweeps, check,
// global PCG finish): every reduction is a workgroup reduction, every
// dependency a workgroup barrier, and one launch serves all G systems, which
// run side by side on separate compute units.  A system's vectors (about
// 37 B per cell) stay in the L2 of the XCD that runs it.
//
// The local system is applied as the stencil restricted to Omega: rows are
// the compacted idx, and the search direction p is zero outside Omega, so
// (B p)_i = sum_{j in Omega} a_ij p_j is the FMA chain of the stencil row in
// ascending column order with zero terms for j outside Omega (bit-identical
// to the gathered B up to the sign of a zero).  Every per-row quantity
// (residual, gradient, expansion bound, Gauss-Seidel update) uses the same
// for_each order as the grid-wide kernels and the oracle; only the dot
// products are summed in another order (a fixed workgroup tree).
//
// The non-symmetric nine-point kind (full storage) is solved by restarted
// GMRES(m) instead of PCG, in the local and the global solve, with the same
// steps as the grid-wide GMRES: classical Gram-Schmidt applied twice, Givens
// rotations on the Hessenberg matrix, right Jacobi preconditioning, a true
// residual at the start of every cycle.  The basis lives in a per-system
// workspace, the Hessenberg matrix and the rotations in LDS.
#pragma once

#include <type_traits>

#include "lcs_gmres.h"
#include "lcs_kernels.h"

namespace lcs {

constexpr int kBatchBlock = 1024;
constexpr int kBatchWaves = kBatchBlock / kWave;
constexpr int32_t kMaxBatch = 65535;          // one workgroup per system on grid x
constexpr int64_t kLdsRows = 7168;             // systems up to this size keep p and q in 112 KB of LDS
constexpr int64_t kMaxBatchN = int64_t(1) << 24;   // cells per system (int32 idx, time)

// per-system result, written by thread 0 of the system's workgroup
struct BatchOut {
    int64_t K;
    int32_t e_rounds, its_local, its_global, n_outer;
    int32_t status, status_local;
    double tau, relres_after_local, relres_final;
};

template <typename real>
__device__ __forceinline__ Stencil5<real> shifted(Stencil5<real> A, int64_t off) {
    A.C += off;
    A.E += off;
    A.N += off;
    return A;
}
template <typename real>
__device__ __forceinline__ Stencil9<real> shifted(Stencil9<real> A, int64_t off) {
    A.C += off;
    A.E += off;
    A.N += off;
    A.NE += off;
    A.NW += off;
    return A;
}
template <typename real>
__device__ __forceinline__ Stencil7<real> shifted(Stencil7<real> A, int64_t off) {
    A.C += off;
    A.E += off;
    A.N += off;
    A.U += off;
    return A;
}

template <typename real>
__device__ __forceinline__ Stencil9N<real> shifted(Stencil9N<real> A, int64_t off) {
    A.a += off;
    return A;
}

template <class S>
struct is_full9 : std::false_type {};
template <typename real>
struct is_full9<Stencil9N<real>> : std::true_type {};

// Branch-free neighbour table of one stencil row.  Slot k runs over the
// row's entries in ascending column order (the order of for_each): column
// j[k] (the row itself where the neighbour is missing), ok[k] whether it
// exists, and coef() loads the coefficients at those clamped positions, so
// every load of a row is unconditional and independent of the others (many
// in flight at once), while the sums skip the missing slots exactly as
// for_each does.
template <class S>
struct RowN;

template <typename real>
struct RowN<Stencil5<real>> {
    static constexpr int NB = 5, kC = 2;
    int32_t j[NB];   // fits: at most 2^24 cells per system
    bool ok[NB];
    __device__ __forceinline__ RowN(const Stencil5<real> &A, int64_t i) {
        const int y = (int)((uint32_t)i / (uint32_t)A.nx), x = (int)i - y * A.nx;
        ok[0] = y > 0;
        ok[1] = x > 0;
        ok[2] = true;
        ok[3] = x < A.nx - 1;
        ok[4] = y < A.ny - 1;
        const int32_t ii = (int32_t)i, nx = A.nx;
        const int32_t d[NB] = {-nx, -1, 0, 1, nx};
#pragma unroll
        for (int k = 0; k < NB; ++k) j[k] = ok[k] ? ii + d[k] : ii;
    }
    __device__ __forceinline__ void coef(const Stencil5<real> &A, int64_t i, double (&a)[NB]) const {
        a[0] = A.N[j[0]];
        a[1] = A.E[j[1]];
        a[2] = A.C[i];
        a[3] = A.E[i];
        a[4] = A.N[i];
    }
};

template <typename real>
struct RowN<Stencil9<real>> {
    static constexpr int NB = 9, kC = 4;
    int32_t j[NB];   // fits: at most 2^24 cells per system
    bool ok[NB];
    __device__ __forceinline__ RowN(const Stencil9<real> &A, int64_t i) {
        const int y = (int)((uint32_t)i / (uint32_t)A.nx), x = (int)i - y * A.nx;
        const bool w = x > 0, e = x < A.nx - 1, s = y > 0, n = y < A.ny - 1;
        ok[0] = s && w;
        ok[1] = s;
        ok[2] = s && e;
        ok[3] = w;
        ok[4] = true;
        ok[5] = e;
        ok[6] = n && w;
        ok[7] = n;
        ok[8] = n && e;
        const int32_t ii = (int32_t)i, nx = A.nx;
        const int32_t d[NB] = {-nx - 1, -nx, -nx + 1, -1, 0, 1, nx - 1, nx, nx + 1};
#pragma unroll
        for (int k = 0; k < NB; ++k) j[k] = ok[k] ? ii + d[k] : ii;
    }
    __device__ __forceinline__ void coef(const Stencil9<real> &A, int64_t i, double (&a)[NB]) const {
        a[0] = A.NE[j[0]];
        a[1] = A.N[j[1]];
        a[2] = A.NW[j[2]];
        a[3] = A.E[j[3]];
        a[4] = A.C[i];
        a[5] = A.E[i];
        a[6] = A.NW[i];
        a[7] = A.N[i];
        a[8] = A.NE[i];
    }
};

template <typename real>
struct RowN<Stencil7<real>> {
    static constexpr int NB = 7, kC = 3;
    int32_t j[NB];   // fits: at most 2^24 cells per system
    bool ok[NB];
    __device__ __forceinline__ RowN(const Stencil7<real> &A, int64_t i) {
        const int64_t pl = (int64_t)A.nx * A.ny;
        const int z = (int)((uint64_t)i / (uint64_t)pl);
        const int r = (int)(i - (int64_t)z * pl);
        const int y = (int)((uint32_t)r / (uint32_t)A.nx), x = r - y * A.nx;
        ok[0] = z > 0;
        ok[1] = y > 0;
        ok[2] = x > 0;
        ok[3] = true;
        ok[4] = x < A.nx - 1;
        ok[5] = y < A.ny - 1;
        ok[6] = z < A.nz - 1;
        const int32_t ii = (int32_t)i, nx = A.nx, p32 = (int32_t)pl;
        const int32_t d[NB] = {-p32, -nx, -1, 0, 1, nx, p32};
#pragma unroll
        for (int k = 0; k < NB; ++k) j[k] = ok[k] ? ii + d[k] : ii;
    }
    __device__ __forceinline__ void coef(const Stencil7<real> &A, int64_t i, double (&a)[NB]) const {
        a[0] = A.U[j[0]];
        a[1] = A.N[j[1]];
        a[2] = A.E[j[2]];
        a[3] = A.C[i];
        a[4] = A.E[i];
        a[5] = A.N[i];
        a[6] = A.U[i];
    }
};

template <typename real>
struct RowN<Stencil9N<real>> {
    static constexpr int NB = 9, kC = 4;
    int32_t j[NB];   // fits: at most 2^24 cells per system
    bool ok[NB];
    __device__ __forceinline__ RowN(const Stencil9N<real> &A, int64_t i) {
        const int y = (int)((uint32_t)i / (uint32_t)A.nx), x = (int)i - y * A.nx;
        const bool w = x > 0, e = x < A.nx - 1, s = y > 0, n = y < A.ny - 1;
        ok[0] = s && w;
        ok[1] = s;
        ok[2] = s && e;
        ok[3] = w;
        ok[4] = true;
        ok[5] = e;
        ok[6] = n && w;
        ok[7] = n;
        ok[8] = n && e;
        const int32_t ii = (int32_t)i, nx = A.nx;
        const int32_t d[NB] = {-nx - 1, -nx, -nx + 1, -1, 0, 1, nx - 1, nx, nx + 1};
#pragma unroll
        for (int k = 0; k < NB; ++k) j[k] = ok[k] ? ii + d[k] : ii;
    }
    // full storage: all nine coefficients of row i sit in row i's slots
    __device__ __forceinline__ void coef(const Stencil9N<real> &A, int64_t i, double (&a)[NB]) const {
#pragma unroll
        for (int k = 0; k < NB; ++k) a[k] = A.a[(int64_t)k * A.n + i];
    }
};

// sum over the row's existing entries in ascending column order:
// acc = fma(sign * a_k, v[j_k], acc)
template <class S, int kSign>
__device__ __forceinline__ double row_fma(const S &A, int64_t i, const double *v, double acc) {
    const RowN<S> R(A, i);
    constexpr int NB = RowN<S>::NB;
    double a[NB], w[NB];
    R.coef(A, i, a);
#pragma unroll
    for (int k = 0; k < NB; ++k) w[k] = v[R.j[k]];
#pragma unroll
    for (int k = 0; k < NB; ++k)
        if (R.ok[k]) acc = fma(kSign > 0 ? a[k] : -a[k], w[k], acc);
    return acc;
}

// Workgroup reduction of NV values (bit k of the Ops mask: value k is a max);
// the result is in every thread, identical in all of them (every thread
// combines the wave results in the same order).
template <int NV, class O>
__device__ __forceinline__ void wg_reduce(double (&v)[NV], O ops) {
    __shared__ double lds[kBatchWaves][NV];
#pragma unroll
    for (int k = 0; k < NV; ++k) v[k] = ops.template reduce_wave<double>(k, v[k]);
    const int w = threadIdx.x / kWave;
    if ((threadIdx.x & (kWave - 1)) == 0) {
#pragma unroll
        for (int k = 0; k < NV; ++k) lds[w][k] = v[k];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        double s = lds[0][k];
#pragma unroll
        for (int q = 1; q < kBatchWaves; ++q) s = ops.template apply<double>(k, s, lds[q][k]);
        v[k] = s;
    }
    __syncthreads();
}

// exclusive workgroup scan of one count per thread; total in every thread
__device__ __forceinline__ int64_t wg_exclusive_scan(int v, int64_t &total) {
    __shared__ int64_t wsum[kBatchWaves];
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    int64_t inc = v;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        const int64_t t = __shfl_up(inc, o, kWave);
        if (lane >= o) inc += t;
    }
    if (lane == kWave - 1) wsum[w] = inc;
    __syncthreads();
    int64_t base = 0, tot = 0;
#pragma unroll
    for (int q = 0; q < kBatchWaves; ++q) {
        if (q < w) base += wsum[q];
        tot += wsum[q];
    }
    __syncthreads();
    total = tot;
    return base + inc - v;
}

// Row t of the active set: idx[t] for a local system, t itself for A.
__device__ __forceinline__ int64_t row_of(const int32_t *idx, int64_t t) { return idx ? idx[t] : t; }

// PCG (standard recurrences, as the oracle's) on the rows of the active set
// (cnt rows: idx[0..cnt) or all of A), Jacobi (kPc 1) or none (kPc 0).
// In: r = residual of the initial sol on the active rows, p zero outside
// them.  sol (d for the local system, x for A) is updated in place; stops at
// ||r|| <= tol or max_iter.  Each row is handled by the same thread in every
// loop, so once the r update has consumed q[i] the slot holds the row's
// preconditioned residual z for the p update.  Returns kStOk, kStNoConv, kStBreakdown or
// kStNonFinite; *its = iterations.
template <class S, int kPc>
__device__ int wg_pcg(const S &A, const int32_t *__restrict__ idx, int64_t cnt, double *r,
                      double *sol, double *p, double *q, double tol, int max_iter, int *its) {
    const int tid = threadIdx.x;
    *its = 0;
    double v[2] = {0.0, 0.0};
    for (int64_t t = tid; t < cnt; t += kBatchBlock) {
        const int64_t i = row_of(idx, t);
        const double ri = r[i];
        const double z = kPc ? ri / A.diag(i) : ri;
        p[i] = z;
        v[0] += ri * ri;
        v[1] += ri * z;
    }
    wg_reduce<2>(v, Ops<0u>());   // its barrier also publishes p
    double rr = v[0], rz = v[1];
    if (!(rr == rr)) return kStNonFinite;
    if (sqrt(rr) <= tol) return kStOk;
    int it = 0;
    while (it < max_iter) {
        double pq[1] = {0.0};
#pragma unroll 4
        for (int64_t t = tid; t < cnt; t += kBatchBlock) {
            const int64_t i = row_of(idx, t);
            const double acc = row_fma<S, 1>(A, i, p, 0.0);
            q[i] = acc;
            pq[0] += p[i] * acc;
        }
        wg_reduce<1>(pq, Ops<0u>());
        if (!(pq[0] > 0.0)) {
            *its = it;
            return pq[0] == pq[0] ? kStBreakdown : kStNonFinite;
        }
        const double alpha = rz / pq[0];
        double w[2] = {0.0, 0.0};
#pragma unroll 4
        for (int64_t t = tid; t < cnt; t += kBatchBlock) {
            const int64_t i = row_of(idx, t);
            sol[i] = fma(alpha, p[i], sol[i]);
            const double ri = fma(-alpha, q[i], r[i]);
            r[i] = ri;
            const double z = kPc ? ri / A.diag(i) : ri;
            q[i] = z;   // q is dead from here on; its slot carries z to the p update
            w[0] += ri * ri;
            w[1] += ri * z;
        }
        wg_reduce<2>(w, Ops<0u>());
        ++it;
        rr = w[0];
        if (!(rr == rr)) {
            *its = it;
            return kStNonFinite;
        }
        if (sqrt(rr) <= tol) {
            *its = it;
            return kStOk;
        }
        const double beta = w[1] / rz;
        rz = w[1];
#pragma unroll 4
        for (int64_t t = tid; t < cnt; t += kBatchBlock) {
            const int64_t i = row_of(idx, t);
            p[i] = fma(beta, p[i], q[i]);
        }
        __syncthreads();
    }
    *its = it;
    return kStNoConv;
}

// The same PCG for systems of at most kLdsRows cells, with the search
// direction p and the product q = A p in LDS (lds[0, kLdsRows) and
// lds[kLdsRows, 2 kLdsRows), indexed by cell; p is zero outside the active
// rows).  The nine gathers of each SpMV row are LDS reads, and the global
// traffic per iteration is the coefficients, the diagonal and the own rows of
// r and sol.  Each row is handled by the same thread in every loop, so after
// the r update the row's preconditioned residual z takes the place of its
// (now dead) q entry and the p update reads only LDS.  Same recurrences and
// FMA orders as wg_pcg.
template <class S, int kPc>
__device__ int wg_pcg_lds(const S &A, const int32_t *__restrict__ idx, int64_t cnt, double *r,
                          double *sol, double *lds, double tol, int max_iter,
                          int *its) {
    using RN = RowN<S>;
    const int tid = threadIdx.x;
    double *p_lds = lds, *q_lds = lds + kLdsRows;
    // the active rows of a local system, copied once into LDS: every row
    // loop below reads its cell index from there instead of global memory
    __shared__ int32_t idx_lds[kLdsRows];
    auto row = [&](int64_t t) -> int64_t { return idx ? (int64_t)idx_lds[t] : t; };
    *its = 0;
    if (idx)
        for (int64_t t = tid; t < cnt; t += kBatchBlock) idx_lds[t] = idx[t];
    for (int64_t i = tid; i < A.n; i += kBatchBlock) p_lds[i] = 0.0;
    __syncthreads();
    double v[2] = {0.0, 0.0};
    for (int64_t t = tid; t < cnt; t += kBatchBlock) {
        const int64_t i = row(t);
        const double ri = r[i];
        const double z = kPc ? ri / A.diag(i) : ri;
        p_lds[i] = z;
        v[0] += ri * ri;
        v[1] += ri * z;
    }
    wg_reduce<2>(v, Ops<0u>());   // its barrier also publishes p_lds
    double rr = v[0], rz = v[1];
    if (!(rr == rr)) return kStNonFinite;
    if (sqrt(rr) <= tol) return kStOk;
    int it = 0;
    while (it < max_iter) {
        double pq[1] = {0.0};
        for (int64_t t = tid; t < cnt; t += kBatchBlock) {
            const int64_t i = row(t);
            const RN Rw(A, i);
            double cf[RN::NB], pv[RN::NB];
            Rw.coef(A, i, cf);
            // every gather first (clamped columns are valid), then the sum
            // with missing slots skipped by a select: the LDS reads of a row
            // issue together instead of one wait per neighbour
#pragma unroll
            for (int s = 0; s < RN::NB; ++s) pv[s] = p_lds[Rw.j[s]];
            double acc = 0.0;
#pragma unroll
            for (int s = 0; s < RN::NB; ++s) {
                const double t = fma(cf[s], pv[s], acc);
                acc = Rw.ok[s] ? t : acc;
            }
            q_lds[i] = acc;   // read back below by this thread only
            pq[0] += p_lds[i] * acc;
        }
        wg_reduce<1>(pq, Ops<0u>());
        if (!(pq[0] > 0.0)) {
            *its = it;
            return pq[0] == pq[0] ? kStBreakdown : kStNonFinite;
        }
        const double alpha = rz / pq[0];
        double w[2] = {0.0, 0.0};
#pragma unroll 2
        for (int64_t t = tid; t < cnt; t += kBatchBlock) {
            const int64_t i = row(t);
            sol[i] = fma(alpha, p_lds[i], sol[i]);
            const double ri = fma(-alpha, q_lds[i], r[i]);
            r[i] = ri;
            const double z = kPc ? ri / A.diag(i) : ri;
            q_lds[i] = z;   // q is dead from here on; its slot carries z to the p update
            w[0] += ri * ri;
            w[1] += ri * z;
        }
        wg_reduce<2>(w, Ops<0u>());
        ++it;
        rr = w[0];
        if (!(rr == rr)) {
            *its = it;
            return kStNonFinite;
        }
        if (sqrt(rr) <= tol) {
            *its = it;
            return kStOk;
        }
        const double beta = w[1] / rz;
        rz = w[1];
#pragma unroll 2
        for (int64_t t = tid; t < cnt; t += kBatchBlock) {
            const int64_t i = row(t);
            p_lds[i] = fma(beta, p_lds[i], q_lds[i]);
        }
        __syncthreads();
    }
    *its = it;
    return kStNoConv;
}

// r = b - A x over all rows (FMA chain, ascending columns); returns ||r||^2
// in every thread.
template <class S>
__device__ double wg_residual(const S &A, const double *__restrict__ b, const double *x, double *r) {
    double v[1] = {0.0};
#pragma unroll 4
    for (int64_t i = threadIdx.x; i < A.n; i += kBatchBlock) {
        const double acc = row_fma<S, -1>(A, i, x, b[i]);
        r[i] = acc;
        v[0] += acc * acc;
    }
    wg_reduce<1>(v, Ops<0u>());
    return v[0];
}

// Global finish: PCG from x with a true-residual check, restarting from the
// current x while the check fails (at most max_outer restarts, max_iter
// iterations in all).  r must hold b - A x on entry.
template <class S, int kPc, bool kLds>
__device__ int wg_global(const S &A, const double *__restrict__ b, double *x, double *r, double *p,
                         double *q, double *p_lds, double tol, int max_iter, int max_outer,
                         int *its_total, int *restarts, double *rr_true) {
    int st = kStOk, total = 0;
    *restarts = 0;
    for (int attempt = 0;; ++attempt) {
        int it = 0;
        if constexpr (kLds)
            st = wg_pcg_lds<S, kPc>(A, nullptr, A.n, r, x, p_lds, tol, max_iter - total, &it);
        else
            st = wg_pcg<S, kPc>(A, nullptr, A.n, r, x, p, q, tol, max_iter - total, &it);
        total += it;
        const double rr = wg_residual(A, b, x, r);
        *rr_true = rr;
        if (st != kStOk) break;
        if (sqrt(rr) <= tol) break;
        if (attempt >= max_outer || total >= max_iter) {
            st = kStNoConv;
            break;
        }
        *restarts += 1;
    }
    *its_total = total;
    return st;
}

// Restarted GMRES(m) of one workgroup on the active rows (cnt rows: idx[0..cnt)
// or all of A), right-preconditioned by Jacobi (kPc 1) or by nothing:
// A M^-1 u = rhs - A sol, sol += M^-1 u.  zb holds a vector supported on the
// active rows (zero elsewhere) for the SpMV gathers, wb the current Arnoldi
// vector (own rows only), V the (m + 1) x n basis.  Every cycle starts from
// the true residual; a cycle ends after m steps, at the estimate meeting tol,
// or at max_iter steps in all.  A cycle that ended on the estimate (or the
// cap) is followed by a check of the true residual, and at most max_outer
// such checks may fail before kStNoConv.  Returns kStOk, kStNoConv,
// kStBreakdown or kStNonFinite; *its = Arnoldi steps, *rr_true = the last
// true ||rhs - A sol||^2.
template <class S, int kPc>
__device__ int wg_gmres(const S &A, const int32_t *__restrict__ idx, int64_t cnt,
                        const double *__restrict__ rhs, double *sol, double *zb, double *wb,
                        double *V, int m, double tol, int max_iter, int max_outer, int *its,
                        int *restarts, double *rr_true) {
    using RN = RowN<S>;
    __shared__ GmState L;   // Hessenberg matrix, rotations, g, y (one per workgroup)
    const int tid = threadIdx.x;
    const int64_t n = A.n;
    int it = 0, outer = 0;
    *its = 0;
    *restarts = 0;
    for (int64_t i = tid; i < n; i += kBatchBlock) zb[i] = 0.0;
    __syncthreads();
    // w = v - A zb over the active rows, v = rhs (residual) or 0 (product)
    auto spmv_rows = [&](bool residual) {
        double acc2 = 0.0;
        for (int64_t t = tid; t < cnt; t += kBatchBlock) {
            const int64_t i = row_of(idx, t);
            const RN Rw(A, i);
            double cf[RN::NB], zv[RN::NB];
            Rw.coef(A, i, cf);
#pragma unroll
            for (int q = 0; q < RN::NB; ++q) zv[q] = zb[Rw.j[q]];
            double acc = residual ? rhs[i] : 0.0;
#pragma unroll
            for (int q = 0; q < RN::NB; ++q) {
                const double tt = residual ? fma(-cf[q], zv[q], acc) : fma(cf[q], zv[q], acc);
                acc = Rw.ok[q] ? tt : acc;
            }
            wb[t] = acc;
            acc2 += acc * acc;
        }
        return acc2;
    };
    bool check_pending = false;
    for (;;) {
        for (int64_t t = tid; t < cnt; t += kBatchBlock) {
            const int64_t i = row_of(idx, t);
            zb[i] = sol[i];
        }
        __syncthreads();
        double v[1] = {spmv_rows(true)};
        wg_reduce<1>(v, Ops<0u>());
        const double beta = sqrt(v[0]);
        *rr_true = v[0];
        if (!(beta == beta)) {
            *its = it;
            return kStNonFinite;
        }
        if (beta <= tol) {
            *its = it;
            return kStOk;
        }
        if (check_pending) {   // the true residual missed tol after the estimate met it
            if (it >= max_iter || outer >= max_outer) {
                *its = it;
                return kStNoConv;
            }
            ++outer;
            *restarts = outer;
        } else if (it >= max_iter) {
            *its = it;
            return kStNoConv;
        }
        for (int64_t t = tid; t < cnt; t += kBatchBlock) V[t] = wb[t] / beta;
        if (tid == 0) {
            L.tol = tol;
            L.done = 0;
            L.status = kStOk;
            gm_column(&L, 0, beta);
        }
        for (int j = 0; j < m && it < max_iter; ++j) {
            const double *vj = V + (int64_t)j * n;
            for (int64_t t = tid; t < cnt; t += kBatchBlock) {
                const int64_t i = row_of(idx, t);
                zb[i] = kPc ? vj[t] / A.diag(i) : vj[t];
            }
            __syncthreads();
            (void)spmv_rows(false);   // w = A M^-1 v_j
            // classical Gram-Schmidt, twice: h = V^T w, w -= V h.  Wave q
            // forms the dot products of basis vectors q, q + 16, ... over all
            // rows and reduces them within the wave: one barrier per pass.
            for (int pass = 0; pass < 2; ++pass) {
                __syncthreads();   // w of the SpMV or of the last update visible
                const int wave = tid / kWave, lane = tid & (kWave - 1);
                for (int c = wave; c <= j; c += kBatchWaves) {
                    const double *vc = V + (int64_t)c * n;
                    double acc = 0.0;
                    for (int64_t t = lane; t < cnt; t += kWave) acc += vc[t] * wb[t];
                    acc = wave_reduce(acc, OpSum());
                    if (lane == 0) L.hc[c] = acc;
                }
                __syncthreads();   // hc of this pass visible
                for (int64_t t = tid; t < cnt; t += kBatchBlock) {
                    double wi = wb[t];
                    for (int q = 0; q <= j; ++q) wi = fma(-L.hc[q], V[(int64_t)q * n + t], wi);
                    wb[t] = wi;
                }
                if (tid == 0) {
                    double *h = L.H + j * kGmLd;
                    for (int q = 0; q <= j; ++q) h[q] = pass == 0 ? L.hc[q] : h[q] + L.hc[q];
                }
                __syncthreads();   // hc read by all before the next pass rewrites it
            }
            double nv[1] = {0.0};
            for (int64_t t = tid; t < cnt; t += kBatchBlock) nv[0] += wb[t] * wb[t];
            wg_reduce<1>(nv, Ops<0u>());
            const double nrm = sqrt(nv[0]);
            ++it;
            if (tid == 0) gm_column(&L, j + 1, nrm);   // rotations, residual estimate
            __syncthreads();
            if (L.done) break;
            double *vn = V + (int64_t)(j + 1) * n;
            for (int64_t t = tid; t < cnt; t += kBatchBlock) vn[t] = wb[t] / nrm;
        }
        if (L.status != kStOk) {
            *its = it;
            return L.status;
        }
        if (tid == 0) {   // back substitution, H y = g on the k completed columns
            const int k = L.k;
            for (int i = k - 1; i >= 0; --i) {
                double acc = L.g[i];
                for (int l = i + 1; l < k; ++l) acc -= L.H[l * kGmLd + i] * L.y[l];
                L.y[i] = acc / L.H[i * kGmLd + i];
            }
        }
        __syncthreads();
        const int k = L.k;
        for (int64_t t = tid; t < cnt; t += kBatchBlock) {
            const int64_t i = row_of(idx, t);
            double u = 0.0;
            for (int q = 0; q < k; ++q) u = fma(L.y[q], V[(int64_t)q * n + t], u);
            if (kPc) u = u / A.diag(i);
            sol[i] += u;
        }
        check_pending = L.done || it >= max_iter;
        __syncthreads();   // L read by all before the next cycle rewrites it
    }
}

struct BatchArgs {
    int64_t coef_stride;   // doubles between consecutive systems' coefficient sets
    int local;             // 0: global PCG only (the baseline); 1: Algorithm 1
    int mode, thresh;      // LCS_MODE_*, LCS_THRESH_* values
    double theta;
    int e_max;
    double eps, tol_local;
    int max_iter, max_outer, n_smooth;
    int restart;           // GMRES restart length (non-symmetric kind)
    double *gm_V;          // GMRES bases: (restart + 1) x n doubles per system
};

// One workgroup per system g = blockIdx.x.  ws: 4 n doubles per system
// (r, p, q, d); stamp: n bytes; idx: n ints.
template <class S, int kPc, bool kLds>
__global__ __launch_bounds__(kBatchBlock) void k_batch_solve(S A0, BatchArgs a,
                                                             const double *__restrict__ b_all,
                                                             double *x_all, double *ws,
                                                             uint8_t *stamp_all, int32_t *idx_all,
                                                             BatchOut *out) {
    const int g = blockIdx.x;
    const S A = shifted(A0, (int64_t)g * a.coef_stride);
    const int64_t n = A.n;
    const int tid = threadIdx.x;
    const double *b = b_all + (int64_t)g * n;
    double *x = x_all + (int64_t)g * n;
    double *r = ws + (int64_t)g * 4 * n, *p = r + n, *q = p + n, *d = q + n;
    double *gm_V = a.gm_V ? a.gm_V + (int64_t)g * (a.restart + 1) * n : nullptr;
    uint8_t *stamp = stamp_all + (int64_t)g * n;
    int32_t *idx = idx_all + (int64_t)g * n;
    BatchOut o{};
    o.status = kStOk;
    __shared__ double lds_buf[kLds ? 2 * kLdsRows : 1];   // p, then q, of the LDS PCG
    double *p_lds = lds_buf;

    // ---- r0 = b - A x0; ||b||^2, ||r0||^2, max |score| (Algorithms 2, 3) ----
    double v[3] = {0.0, 0.0, 0.0};
    using RN = RowN<S>;
    for (int64_t i = tid; i < n; i += kBatchBlock) {
        const double bi = b[i];
        const RN R(A, i);
        double cf[RN::NB], xv[RN::NB];
        R.coef(A, i, cf);
#pragma unroll
        for (int k = 0; k < RN::NB; ++k) xv[k] = x[R.j[k]];
        double acc = bi;
#pragma unroll
        for (int k = 0; k < RN::NB; ++k)
            if (R.ok[k]) acc = fma(-cf[k], xv[k], acc);
        r[i] = acc;
        v[1] += bi * bi;
        v[2] += acc * acc;
        double s = acc;
        if (a.local && a.mode == LCS_MODE_GRADIENT) {
            const double xi = xv[RN::kC];
            double gsum = 0.0;
#pragma unroll
            for (int k = 0; k < RN::NB; ++k)
                if (R.ok[k] && k != RN::kC) gsum += fabs(xi - xv[k]);
            s = gsum;
            q[i] = gsum;   // q holds the gradient score until the local PCG
        }
        const double m = fabs(s);
        v[0] = m > v[0] ? m : v[0];
    }
    wg_reduce<3>(v, Ops<1u>());
    const double bn = sqrt(v[1]);
    const double tol = a.eps * bn;
    const double rr0 = v[2];
    if (!(v[1] == v[1]) || !(rr0 == rr0) || !(v[0] == v[0])) {
        o.status = kStNonFinite;
        if (tid == 0) out[g] = o;
        return;
    }
    double rr = rr0;
    int st_global = kStOk;
    bool need_global = true;

    if (a.local) {
        double tau;
        if (a.thresh == LCS_THRESH_REL_MAX) tau = a.theta * v[0];
        else if (a.thresh == LCS_THRESH_ABS) tau = a.theta;
        else tau = a.theta * bn / sqrt((double)n);
        o.tau = tau;
        if (sqrt(rr0) <= tol) {
            // x0 already meets the criterion: it is the solution
            o.relres_after_local = o.relres_final = bn > 0 ? sqrt(rr0) / bn : sqrt(rr0);
            if (tid == 0) out[g] = o;
            return;
        }
        const bool res_mode = a.mode == LCS_MODE_RESIDUAL;
        // ---- mark (strict >) ----
        for (int64_t i = tid; i < n; i += kBatchBlock)
            stamp[i] = fabs(res_mode ? r[i] : q[i]) > tau ? 1 : 0;
        __syncthreads();
        // ---- synchronous expansion rounds (Algorithm 3, eq. extend-local-condition) ----
        const int ex = res_mode ? a.e_max : 0;
        for (int m = 1; m <= ex; ++m) {
            double added[1] = {0.0};
            for (int64_t j = tid; j < n; j += kBatchBlock) {
                if (stamp[j] != 0) continue;
                const RN R(A, j);
                double cf[RN::NB], xv[RN::NB];
                int sl[RN::NB];
                R.coef(A, j, cf);
#pragma unroll
                for (int k = 0; k < RN::NB; ++k) {
                    xv[k] = x[R.j[k]];
                    sl[k] = stamp[R.j[k]];
                }
                bool nb = false;
                double acc = fabs(r[j]);
#pragma unroll
                for (int k = 0; k < RN::NB; ++k) {
                    if (R.ok[k] && k != RN::kC && sl[k] != 0 && sl[k] <= m) {
                        nb = true;
                        acc += fabs(cf[k] * xv[k]);
                    }
                }
                if (nb && acc > tau) {
                    stamp[j] = (uint8_t)(m + 1);
                    added[0] += 1.0;
                }
            }
            wg_reduce<1>(added, Ops<0u>());
            if (added[0] == 0.0) break;
            o.e_rounds = m;
        }
        // ---- compaction: contiguous chunks per thread, ascending ----
        const int64_t chunk = (n + kBatchBlock - 1) / kBatchBlock;
        const int64_t cb = tid * chunk < n ? tid * chunk : n;
        const int64_t ce = cb + chunk < n ? cb + chunk : n;
        int cnt = 0;
        for (int64_t i = cb; i < ce; ++i) cnt += stamp[i] != 0;
        int64_t K = 0;
        int64_t off = wg_exclusive_scan(cnt, K);
        for (int64_t i = cb; i < ce; ++i)
            if (stamp[i] != 0) idx[off++] = (int32_t)i;
        o.K = K;
        __syncthreads();   // idx is read below by threads that did not write it
        // ---- local PCG on Omega from d = 0, rhs r0_Omega (correction form) ----
        for (int64_t i = tid; i < n; i += kBatchBlock) p[i] = 0.0;
        for (int64_t t = tid; t < K; t += kBatchBlock) d[idx[t]] = 0.0;
        __syncthreads();
        int its = 0;
        if constexpr (is_full9<S>::value) {
            int rst = 0;
            double rr_loc = 0.0;
            double *zb = kLds ? p_lds : p, *wb = kLds ? p_lds + kLdsRows : q;
            o.status_local = wg_gmres<S, kPc>(A, idx, K, r, d, zb, wb, gm_V, a.restart,
                                              a.tol_local * bn, a.max_iter, a.max_outer, &its,
                                              &rst, &rr_loc);
            o.n_outer += rst;
        } else if constexpr (kLds) {
            o.status_local = wg_pcg_lds<S, kPc>(A, idx, K, r, d, p_lds, a.tol_local * bn,
                                                a.max_iter, &its);
        } else {
            o.status_local = wg_pcg<S, kPc>(A, idx, K, r, d, p, q, a.tol_local * bn, a.max_iter,
                                            &its);
        }
        o.its_local = its;
        if (o.status_local == kStBreakdown || o.status_local == kStNonFinite) {
            o.status = o.status_local;
            if (tid == 0) out[g] = o;
            return;
        }
        // ---- assemble x~ (eq. sol-assemble) and smooth ----
        for (int64_t t = tid; t < K; t += kBatchBlock) {
            const int64_t i = idx[t];
            x[i] += d[i];
        }
        __syncthreads();
        for (int sw = 0; sw < a.n_smooth; ++sw)
            for (int c = 0; c < S::kColours; ++c) {
                for (int64_t i = tid; i < n; i += kBatchBlock) {
                    if (A.colour(i) != c) continue;
                    const RN R(A, i);
                    double cf[RN::NB], xv[RN::NB];
                    R.coef(A, i, cf);
#pragma unroll
                    for (int k = 0; k < RN::NB; ++k) xv[k] = x[R.j[k]];
                    double acc = b[i];
#pragma unroll
                    for (int k = 0; k < RN::NB; ++k)
                        if (R.ok[k] && k != RN::kC) acc = fma(-cf[k], xv[k], acc);
                    x[i] = acc / cf[RN::kC];
                }
                __syncthreads();
            }
        // ---- check (eq. rel-res-conv-criteria) ----
        rr = wg_residual(A, b, x, r);
        o.relres_after_local = bn > 0 ? sqrt(rr) / bn : sqrt(rr);
        need_global = !(sqrt(rr) <= tol);
        if (!(rr == rr)) {
            o.status = kStNonFinite;
            if (tid == 0) out[g] = o;
            return;
        }
    }
    if (need_global) {
        // r holds b - A x here (either r0 or the post-smoothing residual)
        int its = 0, restarts = 0;
        if constexpr (is_full9<S>::value) {
            double *zb = kLds ? p_lds : p, *wb = kLds ? p_lds + kLdsRows : q;
            st_global = wg_gmres<S, kPc>(A, nullptr, A.n, b, x, zb, wb, gm_V, a.restart, tol,
                                         a.max_iter, a.max_outer, &its, &restarts, &rr);
        } else {
            st_global = wg_global<S, kPc, kLds>(A, b, x, r, p, q, p_lds, tol, a.max_iter,
                                                a.max_outer, &its, &restarts, &rr);
        }
        o.its_global = its;
        o.n_outer += restarts;
    }
    o.status = st_global;
    o.relres_final = bn > 0 ? sqrt(rr) / bn : sqrt(rr);
    if (tid == 0) out[g] = o;
}

}  // namespace lcs
