// Device-side building blocks of the local character-based solver (gfx950).
//
// Operators visit the stored entries of a row in ascending column order, so
// every per-row sum (residual, SpMV, gradient mimic, expansion bound,
// Gauss-Seidel update) has one fixed rounding sequence.  Reductions are
// deterministic: a fixed wave-shuffle / LDS tree per block, then the last
// block to finish folds the per-block partials in block order.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lcs {

constexpr int kBlock = 256;          // 4 wavefronts of 64
constexpr int kWave = 64;
constexpr int kWaves = kBlock / kWave;
constexpr int kMaxGrid = 1024;       // 4 blocks (16 waves) per CU on 256 CUs
constexpr int kXcds = 8;

// ---------------------------------------------------------------------------
// grid mapping
// ---------------------------------------------------------------------------
// The hardware hands block b to XCD (b mod 8).  Remapping so that each XCD
// owns a contiguous run of chunks keeps stencil neighbours (rows +-nx) in the
// same XCD's L2.
__device__ __forceinline__ int logical_block() {
    const unsigned b = blockIdx.x, g = gridDim.x;
    if (g % kXcds != 0) return (int)b;
    return (int)((b % kXcds) * (g / kXcds) + b / kXcds);
}

struct Chunk {
    int64_t begin, end;
};

__device__ __forceinline__ Chunk my_chunk(int64_t n, int64_t chunk) {
    int64_t lb = logical_block();
    int64_t b = lb * chunk;
    int64_t e = b + chunk;
    if (b > n) b = n;
    if (e > n) e = n;
    return {b, e};
}

// ---------------------------------------------------------------------------
// operators: for_each(i, f) calls f(j, a_ij) over stored entries, ascending j
// ---------------------------------------------------------------------------
template <typename real>
struct Stencil5 {
    const real *C, *E, *N;
    int nx, ny;
    int64_t n;
    template <class F>
    __device__ __forceinline__ void for_each(int64_t i, F &&f) const {
        const int y = (int)((uint32_t)i / (uint32_t)nx);
        const int x = (int)i - y * nx;
        if (y > 0) f(i - nx, N[i - nx]);
        if (x > 0) f(i - 1, E[i - 1]);
        f(i, C[i]);
        if (x < nx - 1) f(i + 1, E[i]);
        if (y < ny - 1) f(i + nx, N[i]);
    }
    __device__ __forceinline__ real diag(int64_t i) const { return C[i]; }
    __device__ __forceinline__ int colour(int64_t i) const {
        const int y = (int)((uint32_t)i / (uint32_t)nx);
        return ((int)i - y * nx + y) & 1;
    }
    static constexpr int kColours = 2;
};

template <typename real>
struct Stencil9 {
    const real *C, *E, *N, *NE, *NW;
    int nx, ny;
    int64_t n;
    template <class F>
    __device__ __forceinline__ void for_each(int64_t i, F &&f) const {
        const int y = (int)((uint32_t)i / (uint32_t)nx);
        const int x = (int)i - y * nx;
        const bool w = x > 0, e = x < nx - 1, s = y > 0, nn = y < ny - 1;
        if (s && w) f(i - nx - 1, NE[i - nx - 1]);
        if (s) f(i - nx, N[i - nx]);
        if (s && e) f(i - nx + 1, NW[i - nx + 1]);
        if (w) f(i - 1, E[i - 1]);
        f(i, C[i]);
        if (e) f(i + 1, E[i]);
        if (nn && w) f(i + nx - 1, NW[i]);
        if (nn) f(i + nx, N[i]);
        if (nn && e) f(i + nx + 1, NE[i]);
    }
    __device__ __forceinline__ real diag(int64_t i) const { return C[i]; }
    // four colours: no two cells of one colour share a nine-point stencil
    __device__ __forceinline__ int colour(int64_t i) const {
        const int y = (int)((uint32_t)i / (uint32_t)nx);
        return (((int)i - y * nx) & 1) + 2 * (y & 1);
    }
    static constexpr int kColours = 4;
};

template <typename real>
struct Stencil7 {
    const real *C, *E, *N, *U;
    int nx, ny, nz;
    int64_t n;
    template <class F>
    __device__ __forceinline__ void for_each(int64_t i, F &&f) const {
        const int64_t pl = (int64_t)nx * ny;
        const int z = (int)((uint64_t)i / (uint64_t)pl);
        const int r = (int)(i - (int64_t)z * pl);
        const int y = (int)((uint32_t)r / (uint32_t)nx);
        const int x = r - y * nx;
        if (z > 0) f(i - pl, U[i - pl]);
        if (y > 0) f(i - nx, N[i - nx]);
        if (x > 0) f(i - 1, E[i - 1]);
        f(i, C[i]);
        if (x < nx - 1) f(i + 1, E[i]);
        if (y < ny - 1) f(i + nx, N[i]);
        if (z < nz - 1) f(i + pl, U[i]);
    }
    __device__ __forceinline__ real diag(int64_t i) const { return C[i]; }
    __device__ __forceinline__ int colour(int64_t i) const {
        const int64_t pl = (int64_t)nx * ny;
        const int z = (int)((uint64_t)i / (uint64_t)pl);
        const int r = (int)(i - (int64_t)z * pl);
        const int y = (int)((uint32_t)r / (uint32_t)nx);
        return (r - y * nx + y + z) & 1;
    }
    static constexpr int kColours = 2;
};

// Restricted system B in CSR (row_ptr int32, ascending columns).
template <typename real>
struct Csr {
    const int32_t *rp, *col;
    const real *val;
    const real *dg;          // diagonal of B
    const uint8_t *clr;      // colour of each row (inherited from the grid)
    int64_t n;
    template <class F>
    __device__ __forceinline__ void for_each(int64_t i, F &&f) const {
        const int32_t e = rp[i + 1];
        for (int32_t k = rp[i]; k < e; ++k) f((int64_t)col[k], val[k]);
    }
    __device__ __forceinline__ real diag(int64_t i) const { return dg[i]; }
    __device__ __forceinline__ int colour(int64_t i) const { return clr[i]; }
};

// ---------------------------------------------------------------------------
// deterministic reductions
// ---------------------------------------------------------------------------
struct OpSum {
    template <typename T>
    __device__ __forceinline__ T operator()(T a, T b) const { return a + b; }
    template <typename T>
    __device__ __forceinline__ static T identity() { return T(0); }
};
struct OpMax {
    template <typename T>
    __device__ __forceinline__ T operator()(T a, T b) const { return a > b ? a : b; }
    template <typename T>
    __device__ __forceinline__ static T identity() { return T(0); }  // used on |values|
};

template <typename T, class Op>
__device__ __forceinline__ T wave_reduce(T v, Op op) {
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) v = op(v, __shfl_xor(v, o, kWave));
    return v;
}

// Block reduction of NV values; the result is valid in thread 0.
template <typename T, int NV, class Ops>
__device__ __forceinline__ void block_reduce(T (&v)[NV], Ops ops) {
    __shared__ T lds[kWaves][NV];
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
#pragma unroll
    for (int k = 0; k < NV; ++k) v[k] = ops.template reduce_wave<T>(k, v[k]);
    if (lane == 0) {
#pragma unroll
        for (int k = 0; k < NV; ++k) lds[w][k] = v[k];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < NV; ++k) {
            T a = lds[0][k];
            for (int q = 1; q < kWaves; ++q) a = ops.template apply<T>(k, a, lds[q][k]);
            v[k] = a;
        }
    }
    __syncthreads();
}

// Per-value operator table: bit k of kMaxMask set -> value k is a max.
template <unsigned kMaxMask>
struct Ops {
    template <typename T>
    __device__ __forceinline__ T apply(int k, T a, T b) const {
        return ((kMaxMask >> k) & 1u) ? (a > b ? a : b) : a + b;
    }
    template <typename T>
    __device__ __forceinline__ T reduce_wave(int k, T v) const {
        if ((kMaxMask >> k) & 1u) return wave_reduce(v, OpMax());
        return wave_reduce(v, OpSum());
    }
};

// Producer side: this block's reduced values go to part[k * gridDim.x + b]
// with plain stores.  There is no cross-block handshake inside a kernel: the
// consumer is the next kernel on the stream, and the kernel boundary makes the
// partials visible (on a multi-XCD part an in-kernel agent-scope fence per
// block would write back and invalidate the XCD's L2 every time).
template <typename T, int NV, class O>
__device__ __forceinline__ void write_partials(T (&v)[NV], O ops, T *part) {
    block_reduce<T, NV>(v, ops);
    if (threadIdx.x == 0) {
        const unsigned g = gridDim.x;
#pragma unroll
        for (int k = 0; k < NV; ++k) part[(size_t)k * g + blockIdx.x] = v[k];
    }
}

// Consumer side: fold the g partials of the producing kernel in a fixed order
// (strided per thread, then the block tree).  Every block that calls this
// gets bit-identical totals, valid in all of its threads.
template <typename T, int NV, class O>
__device__ __forceinline__ void read_partials(const T *part, int g, O ops, T (&tot)[NV]) {
    __shared__ T res[NV];
    T a[NV];
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        a[k] = T(0);
        for (int b = threadIdx.x; b < g; b += kBlock) {
            const T p = part[(size_t)k * g + b];
            a[k] = (b == (int)threadIdx.x) ? p : ops.template apply<T>(k, a[k], p);
        }
    }
    block_reduce<T, NV>(a, ops);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < NV; ++k) res[k] = a[k];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < NV; ++k) tot[k] = res[k];
    __syncthreads();
}

// exclusive prefix of integer block counts: sum of cnt[0..upto) in every
// thread, plus the grand total of cnt[0..g)
__device__ __forceinline__ void block_prefix_of_counts(const int32_t *cnt, int g, int upto,
                                                       int &before, int &total) {
    __shared__ int red[2][kWaves];
    int a = 0, t = 0;
    for (int b = threadIdx.x; b < g; b += kBlock) {
        const int c = cnt[b];
        t += c;
        if (b < upto) a += c;
    }
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) {
        a += __shfl_xor(a, o, kWave);
        t += __shfl_xor(t, o, kWave);
    }
    const int w = threadIdx.x / kWave;
    if ((threadIdx.x & (kWave - 1)) == 0) {
        red[0][w] = a;
        red[1][w] = t;
    }
    __syncthreads();
    int sa = 0, st = 0;
#pragma unroll
    for (int q = 0; q < kWaves; ++q) {
        sa += red[0][q];
        st += red[1][q];
    }
    __syncthreads();
    before = sa;
    total = st;
}

}  // namespace lcs
