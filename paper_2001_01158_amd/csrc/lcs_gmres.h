// Restarted GMRES(m) for the non-symmetric operators (the paper's Krylov
// method, Section 3), right-preconditioned by Jacobi or by nothing:
// A M^-1 u = r0, x = x0 + M^-1 u.
//
// One Arnoldi step j is three wide launches and three one-block folds, with
// no host round trip:
//   k_gm_arnoldi  v_j = w_j / ||w_j|| (stored; the SpMV recomputes it at the
//                 neighbours from the raw w_j); w = A M^-1 v_j; partial dots
//                 V^T w (first Gram-Schmidt pass)
//   k_gm_fold_h   h = V^T w into the state (one block per value); Hessenberg
//                 column j = h
//   k_gm_cgs(0)   w -= V h; partial dots V^T w (second pass)
//   k_gm_fold_h   h2 into the state; column j += h2
//   k_gm_cgs(1)   w -= V h2; partial ||w||^2
//   k_gm_fold_n   ||w||; one thread finishes column j (previous Givens
//                 rotations, a new one, the residual estimate |g_{j+1}|)
// Classical Gram-Schmidt applied twice (CGS2) is as stable as modified
// Gram-Schmidt and needs one reduction per pass instead of one per basis
// vector; in exact arithmetic its Hessenberg matrix is the one the oracle's
// modified Gram-Schmidt builds.  The folds run in their own small grids so that the wide
// kernels, which stream the basis, carry no fold of their own and can use a
// grid large enough to keep HBM busy.  After the cycle one block
// back-substitutes y, and k_gm_update adds M^-1 V y to x.  Kernels read a
// done flag written by an earlier kernel and exit at once after
// convergence, so a cycle can be enqueued in chunks.
#pragma once

#include "lcs_kernels.h"

namespace lcs {

constexpr int kMaxRestart = 64;
constexpr int kGmLd = kMaxRestart + 1;   // leading dimension of H
constexpr int kGmGrid = 1024;            // blocks of the GMRES vector kernels
constexpr int kGmPartVals = kMaxRestart + 1 + 8;   // per-block values of a dot pass (padded)

struct GmState {
    double tol;       // absolute tolerance on the residual estimate
    double res;       // |g_k| after the last completed column
    int32_t done;     // estimate met tol, zero residual, or an exact breakdown
    int32_t k;        // columns completed in this cycle
    int32_t status;   // kStOk, kStBreakdown or kStNonFinite
    int32_t pad;
    double nrm;       // ||w_j|| of the current step (set by k_gm_fold_n)
    double hc[kMaxRestart + 1];   // coefficients of the current Gram-Schmidt pass
    double cs[kMaxRestart], sn[kMaxRestart], g[kMaxRestart + 1], y[kMaxRestart];
    double H[kGmLd * kMaxRestart];   // column c at H[c * kGmLd + i]
};

// Finish Hessenberg column j-1 with its subdiagonal nrm = ||w_j|| (j >= 1),
// or start the cycle with beta = nrm (j == 0).  One thread.
__device__ __forceinline__ void gm_column(GmState *st, int j, double nrm) {
    if (!(nrm == nrm)) {
        st->status = kStNonFinite;
        st->done = 1;
        return;
    }
    if (j == 0) {
        st->g[0] = nrm;
        st->res = nrm;
        st->k = 0;
        if (nrm <= st->tol) st->done = 1;
        return;
    }
    const int c = j - 1;
    double *h = st->H + c * kGmLd;
    h[j] = nrm;
    for (int i = 0; i < c; ++i) {
        const double t = st->cs[i] * h[i] + st->sn[i] * h[i + 1];
        h[i + 1] = -st->sn[i] * h[i] + st->cs[i] * h[i + 1];
        h[i] = t;
    }
    const double a = h[c], b = h[j];
    const double den = sqrt(a * a + b * b);
    if (!(den > 0.0)) {   // A M^-1 v_c = 0: singular operator
        st->status = den == den ? kStBreakdown : kStNonFinite;
        st->done = 1;
        return;
    }
    const double cs = a / den, sn = b / den;
    st->cs[c] = cs;
    st->sn[c] = sn;
    h[c] = den;
    h[j] = 0.0;
    st->g[j] = -sn * st->g[c];
    st->g[c] = cs * st->g[c];
    st->res = fabs(st->g[j]);
    st->k = j;
    if (st->res <= st->tol || nrm == 0.0) st->done = 1;
}

// Partial dots of V_0..V_{cnt-1} with w over this block's rows, eight
// vectors per sweep of the rows.
template <class Op>
__device__ __forceinline__ void gm_dots(const Op &A, const double *V, int64_t ld, const double *w,
                                        int cnt, double *part) {
    for (int v0 = 0; v0 < cnt; v0 += 8) {
        double acc[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
        for (auto Wk = walk<0>(A); Wk.valid(); Wk.advance()) {
            typename Op::Unit U;
            Wk.geom(A, U);
            const double wi = w[U.i0];
#pragma unroll
            for (int q = 0; q < 8; ++q)
                if (v0 + q < cnt) acc[q] += V[(int64_t)(v0 + q) * ld + U.i0] * wi;
        }
        write_partials<double, 8>(acc, Ops<0u>(), part + (size_t)v0 * gridDim.x);
    }
}

// r = rhs - A x (x == nullptr: x = 0) into W0; partial ||r||^2; resets the
// cycle state.
template <class Op>
__global__ __launch_bounds__(kBlock) void k_gm_init(Op A, const double *__restrict__ rhs,
                                                    const double *__restrict__ x, double *W0,
                                                    double *part, GmState *st,
                                                    const double *tol_base, double tol_factor) {
    static_assert(Op::V == 1, "GMRES vectors are walked one row per unit");
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        st->done = 0;
        st->k = 0;
        st->status = kStOk;
        st->res = 0.0;
        st->tol = tol_factor * *tol_base;
    }
    double v[1] = {0.0};
    for (auto W = walk<1>(A); W.valid(); W.advance()) {
        typename Op::Unit U;
        double r;
        if (x) {
            W.load(A, U);
            double xv[Op::NB][1];
            W.template gather<0>(A, U, x, xv);
            double acc = rhs[U.i0];
#pragma unroll
            for (int s = 0; s < Op::NB; ++s)
                if (A.valid(U, s, 0)) acc = fma(-U.a[s][0], xv[s][0], acc);
            r = acc;
        } else {
            W.geom(A, U);
            r = rhs[U.i0];
        }
        W0[U.i0] = r;
        v[0] += r * r;
    }
    write_partials<double, 1>(v, Ops<0u>(), part);
}

// ||w_j|| from the partials of k_gm_init (j = 0) or k_gm_cgs(1); one thread
// starts the cycle (j = 0) or finishes column j-1.  One block.
__global__ __launch_bounds__(kBlock) void k_gm_fold_n(const double *part, int g, int j, GmState *st) {
    if (st->done) return;
    double nn[1];
    read_partials<double, 1>(part, g, Ops<0u>(), nn);
    if (threadIdx.x == 0) {
        const double nrm = sqrt(nn[0]);
        st->nrm = nrm;
        gm_column(st, j, nrm);
    }
}

// The j+1 dots of a Gram-Schmidt pass into st->hc; pass 0 sets Hessenberg
// column j, pass 1 adds to it.  Grid j+1: block v folds value v.
__global__ __launch_bounds__(kBlock) void k_gm_fold_h(const double *part, int g, int j, GmState *st,
                                                      int pass) {
    if (st->done) return;
    const int v = blockIdx.x;
    double t[1];
    read_partials<double, 1>(part + (size_t)v * g, g, Ops<0u>(), t);
    if (threadIdx.x == 0) {
        double *h = st->H + j * kGmLd;
        st->hc[v] = t[0];
        h[v] = pass == 0 ? t[0] : h[v] + t[0];
    }
}

// Arnoldi step j: v_j = Wc / ||w_j|| (own rows stored; recomputed at the
// neighbours), Wn = A M^-1 v_j, partial dots V_0..V_j . Wn.
template <class Op, int kPc>
__global__ __launch_bounds__(kBlock) void k_gm_arnoldi(Op A, double *V, int64_t ld,
                                                       const double *__restrict__ Wc, double *Wn,
                                                       int j, double *part_h, const GmState *st) {
    if (st->done) return;
    const double nrm = st->nrm;
    double *Vj = V + (int64_t)j * ld;
    const double *dg = A.diag_ptr();
    for (auto W = walk<1>(A); W.valid(); W.advance()) {
        typename Op::Unit U;
        W.load(A, U);
        double wv[Op::NB][1], dv[Op::NB][1];
        W.template gather<0>(A, U, Wc, wv);
        if (kPc) A.gather(U, dg, dv);
        double acc = 0.0, own = 0.0;
#pragma unroll
        for (int s = 0; s < Op::NB; ++s) {
            if (!A.valid(U, s, 0)) continue;
            const double v = wv[s][0] / nrm;
            const double z = kPc ? v / dv[s][0] : v;
            acc = fma(U.a[s][0], z, acc);
            if (A.is_diag(U, s, 0)) own = v;
        }
        Vj[U.i0] = own;
        Wn[U.i0] = acc;
    }
    gm_dots(A, V, ld, Wn, j + 1, part_h);
}

// Gram-Schmidt pass `pass` (0 or 1) of step j: Wn -= V hc; pass 0 writes the
// next dots, pass 1 ||Wn||^2.
template <class Op>
__global__ __launch_bounds__(kBlock) void k_gm_cgs(Op A, const double *__restrict__ V, int64_t ld,
                                                   double *Wn, int j, double *part_out,
                                                   const GmState *st, int pass) {
    if (st->done) return;
    __shared__ double hs[kMaxRestart + 1];
    for (int t = threadIdx.x; t <= j; t += kBlock) hs[t] = st->hc[t];
    __syncthreads();
    double v[1] = {0.0};
    for (auto Wk = walk<0>(A); Wk.valid(); Wk.advance()) {
        typename Op::Unit U;
        Wk.geom(A, U);
        double w = Wn[U.i0];
#pragma unroll 8
        for (int q = 0; q <= j; ++q) w = fma(-hs[q], V[(int64_t)q * ld + U.i0], w);
        Wn[U.i0] = w;
        v[0] += w * w;
    }
    if (pass == 0) gm_dots(A, V, ld, Wn, j + 1, part_out);
    else write_partials<double, 1>(v, Ops<0u>(), part_out);
}

// Back substitution H y = g over the k completed columns (row by row,
// ascending l in each sum, as the oracle).  The triangle and g are staged in
// LDS first, so the one thread that substitutes reads no global memory.
__global__ __launch_bounds__(kBlock) void k_gm_finish(GmState *st) {
    __shared__ double Hs[kMaxRestart * kMaxRestart];
    __shared__ double gs[kMaxRestart], ys[kMaxRestart];
    if (st->status != kStOk) return;
    const int k = st->k;
    for (int t = threadIdx.x; t < k * k; t += kBlock) {
        const int c = t / k, i = t - c * k;
        Hs[c * kMaxRestart + i] = st->H[c * kGmLd + i];
    }
    for (int t = threadIdx.x; t < k; t += kBlock) gs[t] = st->g[t];
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int i = k - 1; i >= 0; --i) {
            double acc = gs[i];
            for (int l = i + 1; l < k; ++l) acc -= Hs[l * kMaxRestart + i] * ys[l];
            ys[i] = acc / Hs[i * kMaxRestart + i];
        }
    }
    __syncthreads();
    for (int t = threadIdx.x; t < k; t += kBlock) st->y[t] = ys[t];
}

// x += M^-1 (V_0..V_{k-1} y)
template <class Op, int kPc>
__global__ __launch_bounds__(kBlock) void k_gm_update(Op A, const double *__restrict__ V, int64_t ld,
                                                      double *x, const GmState *st) {
    const int k = st->k;
    if (k == 0 || st->status != kStOk) return;
    for (auto Wk = walk<0>(A); Wk.valid(); Wk.advance()) {
        typename Op::Unit U;
        Wk.geom(A, U);
        double u = 0.0;
#pragma unroll 8
        for (int q = 0; q < k; ++q) u = fma(st->y[q], V[(int64_t)q * ld + U.i0], u);
        if (kPc) {
            double d[1];
            A.diag(U, d);
            u = u / d[0];
        }
        x[U.i0] += u;
    }
}

}  // namespace lcs
