// General sparse input.  A matrix given in CSR (ascending columns within a
// row, diagonal stored) is checked and copied, once per library call, into
// the column-major ELL layout of the restricted systems, with the width
// rounded up to 5, 7, 9 or 16.  Every step of the path (scores and marking of
// Algorithms 2 and 3, the gather of B = A[Omega, Omega] of eq. BEFC, PCG,
// Gauss-Seidel sweeps) then runs on the same row-per-lane ELL operator as
// the restricted systems: slot s of consecutive rows is contiguous, so the
// loads of a wavefront coalesce and need no row-pointer indirection.
#pragma once

#include "lcs_device.h"

namespace lcs {

constexpr int kCsrMaxRow = 64;

// error bits of the structure check
enum : int32_t {
    kCsrBadPtr = 1,     // row_ptr not non-decreasing within [0, nnz]
    kCsrLong = 2,       // a row with more than kCsrMaxRow entries
    kCsrCol = 4,        // a column outside [0, N)
    kCsrOrder = 8,      // columns not strictly ascending within a row
    kCsrNoDiag = 16,    // a row without its diagonal entry
    kCsrColour = 32,    // a colour >= n_colours, or one colour on both ends of an entry
    kCsrEnds = 64,      // row_ptr[0] != 0 or row_ptr[N] != nnz
    kCsrEmpty = 128,    // a row without entries
    kCsrNonFinite = 256,  // a NaN or infinite value
    kCsrBadDiag = 512     // a diagonal <= 0 (symmetric: not SPD) or == 0 (non-symmetric)
};

// Structure and value check and longest row.  flags[0] |= error bits,
// flags[1] = max(flags[1], longest row); both start at zero.  Reads of col,
// val and clr stay inside the ranges the row pointers claim only after those
// pointers passed their own check.  Every value must be finite, and the
// diagonal positive (symmetric input, which PCG needs SPD) or nonzero
// (non-symmetric input, for the Jacobi scaling).
__global__ __launch_bounds__(kBlock) void k_csr_check(const int32_t *__restrict__ rp,
                                                      const int32_t *__restrict__ col,
                                                      const double *__restrict__ val, int64_t n,
                                                      int64_t nnz, const uint8_t *__restrict__ clr,
                                                      int ncol, int nonsym, int32_t *flags) {
    int32_t err = 0, longest = 0;
    for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kBlock) {
        const int64_t a = rp[i], b = rp[i + 1];
        if (a < 0 || b < a || b > nnz) {
            err |= kCsrBadPtr;
            continue;
        }
        const int64_t len = b - a;
        if (len == 0) err |= kCsrEmpty;
        if (len > kCsrMaxRow) {
            err |= kCsrLong;
            longest = kCsrMaxRow + 1;
            continue;
        }
        longest = (int32_t)len > longest ? (int32_t)len : longest;
        const int ci = clr ? (int)clr[i] : 0;
        if (clr && ci >= ncol) err |= kCsrColour;
        bool diag = false;
        int64_t prev = -1;
        for (int64_t k = a; k < b; ++k) {
            const int64_t c = col[k];
            const double v = val[k];
            const bool finite = fabs(v) <= 1.7976931348623157e308;
            if (!finite) err |= kCsrNonFinite;
            if (c < 0 || c >= n) {
                err |= kCsrCol;
                continue;
            }
            if (c <= prev) err |= kCsrOrder;
            prev = c;
            if (c == i) {
                diag = true;
                if (finite && (nonsym ? v == 0.0 : v <= 0.0)) err |= kCsrBadDiag;
            } else if (clr && (int)clr[c] == ci) {
                err |= kCsrColour;
            }
        }
        if (!diag) err |= kCsrNoDiag;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0 && (rp[0] != 0 || (int64_t)rp[n] != nnz)) err |= kCsrEnds;
    __shared__ int32_t se[kBlock], sl[kBlock];
    se[threadIdx.x] = err;
    sl[threadIdx.x] = longest;
    __syncthreads();
    for (int o = kBlock / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) {
            se[threadIdx.x] |= se[threadIdx.x + o];
            sl[threadIdx.x] = sl[threadIdx.x + o] > sl[threadIdx.x] ? sl[threadIdx.x + o] : sl[threadIdx.x];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        if (se[0]) atomicOr(&flags[0], se[0]);
        if (sl[0]) atomicMax(&flags[1], sl[0]);
    }
}

// CSR -> column-major ELL of width W (members in CSR order, then col = -1,
// val = 0), the diagonal after the W value columns (eval[W n + i]) and the
// colour of each row (0 without a colouring).  Runs only after k_csr_check
// found no error, so every row holds 1..W entries inside [0, nnz).
template <int W>
__global__ __launch_bounds__(kBlock) void k_csr_to_ell(const int32_t *__restrict__ rp,
                                                       const int32_t *__restrict__ col,
                                                       const double *__restrict__ val, int64_t n,
                                                       const uint8_t *__restrict__ clr,
                                                       int32_t *__restrict__ ecol,
                                                       double *__restrict__ eval,
                                                       uint8_t *__restrict__ eclr) {
    for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kBlock) {
        const int64_t a = rp[i], b = rp[i + 1];
        double d = 0.0;
#pragma unroll
        for (int s = 0; s < W; ++s) {
            const int64_t k = a + s;
            if (k < b) {
                const int32_t c = col[k];
                const double v = val[k];
                ecol[s * n + i] = c;
                eval[s * n + i] = v;
                if (c == i) d = v;
            } else {
                ecol[s * n + i] = -1;
                eval[s * n + i] = 0.0;
            }
        }
        eval[(int64_t)W * n + i] = d;
        eclr[i] = clr ? clr[i] : (uint8_t)0;
    }
}

// The ELL copy as a unit operator that streams: column indices and values
// are read, and results written, with non-temporal loads and stores.  For
// matrices whose pass exceeds the last-level cache, as the stencil kernels
// do in that case; the gathers of x keep ordinary loads.
template <typename real_, int NB_>
struct UEllStream : UEll<real_, NB_> {
    using Base = UEll<real_, NB_>;
    using Unit = typename Base::Unit;
    __device__ __forceinline__ void load(Unit &U, int64_t u) const {
        U.i0 = u;
#pragma unroll
        for (int s = 0; s < NB_; ++s) {
            U.c[s] = __builtin_nontemporal_load(this->col + s * this->n + u);
            U.a[s][0] = __builtin_nontemporal_load(this->val + s * this->n + u);
        }
    }
    template <typename T>
    __device__ __forceinline__ void put(const Unit &U, T *__restrict__ p, const T (&o)[1]) const {
        __builtin_nontemporal_store(o[0], p + U.i0);
    }
};

template <typename real, int NB>
constexpr bool is_ell<UEllStream<real, NB>> = true;

// Row operator over the ELL copy (the marking rounds and the gather of B):
// the members of row i in ascending column order.
template <typename real, int W>
struct EllRows {
    const int32_t *col;
    const real *val;
    const real *dg;
    const uint8_t *clr;
    int64_t n;
    template <class F>
    __device__ __forceinline__ void for_each(int64_t i, F &&f) const {
#pragma unroll
        for (int s = 0; s < W; ++s) {
            const int32_t c = col[s * n + i];
            if (c >= 0) f((int64_t)c, val[s * n + i]);
        }
    }
    __device__ __forceinline__ real diag(int64_t i) const { return dg[i]; }
    __device__ __forceinline__ int colour(int64_t i) const { return clr[i]; }
};

}  // namespace lcs
