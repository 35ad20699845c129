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
// unit operators: the grid-sized kernels walk "units" — a strip of V
// consecutive cells of one grid row for the stencils (vector loads of every
// coefficient array, halo cells by scalar loads), or one row of the
// restricted matrix in column-major ELL form.  For each cell k of a unit,
// slots s = 0..NB-1 enumerate the stored entries in ascending column order
// (a[s][k] the coefficient, gather() the neighbour values), so every per-cell
// sum has the same rounding sequence as the scalar for_each above.
// ---------------------------------------------------------------------------
template <typename T, int V>
__device__ __forceinline__ void vld(const T *__restrict__ p, T (&o)[V]) {
    if constexpr (V == 1) {
        o[0] = p[0];
    } else {
        typedef T vt __attribute__((ext_vector_type(V)));
        const vt t = *reinterpret_cast<const vt *>(p);
#pragma unroll
        for (int k = 0; k < V; ++k) o[k] = t[k];
    }
}
template <typename T, int V>
__device__ __forceinline__ void vst(T *__restrict__ p, const T (&o)[V]) {
    if constexpr (V == 1) {
        p[0] = o[0];
    } else {
        typedef T vt __attribute__((ext_vector_type(V)));
        vt t;
#pragma unroll
        for (int k = 0; k < V; ++k) t[k] = o[k];
        *reinterpret_cast<vt *>(p) = t;
    }
}

// XCD bands: units [0, nu) are cut into 8 contiguous bands, band b%8 served
// by the blocks b%8 == const (the hardware places block b on XCD b mod 8);
// inside a band the blocks stride together, so rows y-1, y, y+1 are read by
// one XCD close in time and stay in its L2.  gridDim.x is a multiple of 8.
struct Band {
    int64_t u, end, step;
};
__device__ __forceinline__ Band my_band(int64_t nu) {
    const int64_t per = gridDim.x / kXcds;
    const int64_t xcd = blockIdx.x % kXcds, pos = blockIdx.x / kXcds;
    const int64_t band = (nu + kXcds - 1) / kXcds;
    int64_t b0 = xcd * band, b1 = b0 + band;
    if (b1 > nu) b1 = nu;
    return {b0 + pos * kBlock + threadIdx.x, b1, per * kBlock};
}

template <typename real_, int V_>
struct U5 {
    using real = real_;
    static constexpr int V = V_, NB = 5, kC = 2;
    const real *C, *E, *N;
    int nx, ny;
    int64_t n;
    struct Unit {
        int64_t i0;
        int x0, y;
        real a[NB][V];
    };
    __host__ __device__ int64_t units() const { return n / V; }
    __device__ __forceinline__ void geom(Unit &U, int64_t u) const {
        U.i0 = u * V;
        U.y = (int)((uint64_t)U.i0 / (uint64_t)nx);
        U.x0 = (int)(U.i0 - (int64_t)U.y * nx);
    }
    __device__ __forceinline__ void load(Unit &U, int64_t u) const {
        geom(U, u);
        const int64_t i0 = U.i0;
        real c[V], e[V], nn[V], ns[V];
        vld<real, V>(C + i0, c);
        vld<real, V>(E + i0, e);
        vld<real, V>(N + i0, nn);
        if (U.y > 0) vld<real, V>(N + i0 - nx, ns);
        else
#pragma unroll
            for (int k = 0; k < V; ++k) ns[k] = real(0);
        const real ew = U.x0 > 0 ? E[i0 - 1] : real(0);
#pragma unroll
        for (int k = 0; k < V; ++k) {
            U.a[0][k] = ns[k];
            U.a[1][k] = k == 0 ? ew : e[k > 0 ? k - 1 : 0];
            U.a[2][k] = c[k];
            U.a[3][k] = e[k];
            U.a[4][k] = nn[k];
        }
    }
    __device__ __forceinline__ bool valid(const Unit &U, int s, int k) const {
        switch (s) {
        case 0: return U.y > 0;
        case 1: return U.x0 + k > 0;
        case 2: return true;
        case 3: return U.x0 + k < nx - 1;
        default: return U.y < ny - 1;
        }
    }
    __device__ __forceinline__ bool is_diag(const Unit &, int s, int) const { return s == kC; }
    template <typename T>
    __device__ __forceinline__ void gather(const Unit &U, const T *__restrict__ v, T (&o)[NB][V]) const {
        const int64_t i0 = U.i0;
        T c[V], sv[V], nv[V];
        vld<T, V>(v + i0, c);
        if (U.y > 0) vld<T, V>(v + i0 - nx, sv);
        else
#pragma unroll
            for (int k = 0; k < V; ++k) sv[k] = T(0);
        if (U.y < ny - 1) vld<T, V>(v + i0 + nx, nv);
        else
#pragma unroll
            for (int k = 0; k < V; ++k) nv[k] = T(0);
        const T w = U.x0 > 0 ? v[i0 - 1] : T(0);
        const T e = U.x0 + V < nx ? v[i0 + V] : T(0);
#pragma unroll
        for (int k = 0; k < V; ++k) {
            o[0][k] = sv[k];
            o[1][k] = k == 0 ? w : c[k > 0 ? k - 1 : 0];
            o[2][k] = c[k];
            o[3][k] = k == V - 1 ? e : c[k < V - 1 ? k + 1 : 0];
            o[4][k] = nv[k];
        }
    }
    __device__ __forceinline__ int colour(const Unit &U, int k) const { return (U.x0 + k + U.y) & 1; }
    __device__ __forceinline__ void diag(const Unit &U, real (&d)[V]) const { vld<real, V>(C + U.i0, d); }
    __device__ __forceinline__ const real *diag_ptr() const { return C; }
    template <typename T>
    __device__ __forceinline__ void own(const Unit &U, const T *__restrict__ p, T (&o)[V]) const {
        vld<T, V>(p + U.i0, o);
    }
    template <typename T>
    __device__ __forceinline__ void put(const Unit &U, T *__restrict__ p, const T (&o)[V]) const {
        vst<T, V>(p + U.i0, o);
    }
};

template <typename real_, int V_>
struct U9 {
    using real = real_;
    static constexpr int V = V_, NB = 9, kC = 4;
    const real *C, *E, *N, *NE, *NW;
    int nx, ny;
    int64_t n;
    struct Unit {
        int64_t i0;
        int x0, y;
        real a[NB][V];
    };
    __host__ __device__ int64_t units() const { return n / V; }
    __device__ __forceinline__ void geom(Unit &U, int64_t u) const {
        U.i0 = u * V;
        U.y = (int)((uint64_t)U.i0 / (uint64_t)nx);
        U.x0 = (int)(U.i0 - (int64_t)U.y * nx);
    }
    __device__ __forceinline__ void load(Unit &U, int64_t u) const {
        geom(U, u);
        const int64_t i0 = U.i0;
        const bool s = U.y > 0, w = U.x0 > 0, e = U.x0 + V < nx;
        real c[V], ee[V], nn[V], ne[V], nw[V], ns[V], nes[V], nws[V];
        vld<real, V>(C + i0, c);
        vld<real, V>(E + i0, ee);
        vld<real, V>(N + i0, nn);
        vld<real, V>(NE + i0, ne);
        vld<real, V>(NW + i0, nw);
        if (s) {
            vld<real, V>(N + i0 - nx, ns);
            vld<real, V>(NE + i0 - nx, nes);
            vld<real, V>(NW + i0 - nx, nws);
        } else {
#pragma unroll
            for (int k = 0; k < V; ++k) ns[k] = nes[k] = nws[k] = real(0);
        }
        const real ew = w ? E[i0 - 1] : real(0);
        const real nesw = (s && w) ? NE[i0 - nx - 1] : real(0);
        const real nwse = (s && e) ? NW[i0 - nx + V] : real(0);
#pragma unroll
        for (int k = 0; k < V; ++k) {
            U.a[0][k] = k == 0 ? nesw : nes[k > 0 ? k - 1 : 0];
            U.a[1][k] = ns[k];
            U.a[2][k] = k == V - 1 ? nwse : nws[k < V - 1 ? k + 1 : 0];
            U.a[3][k] = k == 0 ? ew : ee[k > 0 ? k - 1 : 0];
            U.a[4][k] = c[k];
            U.a[5][k] = ee[k];
            U.a[6][k] = nw[k];
            U.a[7][k] = nn[k];
            U.a[8][k] = ne[k];
        }
    }
    __device__ __forceinline__ bool valid(const Unit &U, int s, int k) const {
        const bool w = U.x0 + k > 0, e = U.x0 + k < nx - 1, so = U.y > 0, no = U.y < ny - 1;
        switch (s) {
        case 0: return so && w;
        case 1: return so;
        case 2: return so && e;
        case 3: return w;
        case 4: return true;
        case 5: return e;
        case 6: return no && w;
        case 7: return no;
        default: return no && e;
        }
    }
    __device__ __forceinline__ bool is_diag(const Unit &, int s, int) const { return s == kC; }
    template <typename T>
    __device__ __forceinline__ void row3(const Unit &U, const T *__restrict__ v, int64_t base, bool on,
                                         T (&r)[V + 2]) const {
        if (on) {
            T m[V];
            vld<T, V>(v + base, m);
#pragma unroll
            for (int k = 0; k < V; ++k) r[k + 1] = m[k];
            r[0] = U.x0 > 0 ? v[base - 1] : T(0);
            r[V + 1] = U.x0 + V < nx ? v[base + V] : T(0);
        } else {
#pragma unroll
            for (int k = 0; k < V + 2; ++k) r[k] = T(0);
        }
    }
    template <typename T>
    __device__ __forceinline__ void gather(const Unit &U, const T *__restrict__ v, T (&o)[NB][V]) const {
        T rs[V + 2], rc[V + 2], rn[V + 2];
        row3(U, v, U.i0 - nx, U.y > 0, rs);
        row3(U, v, U.i0, true, rc);
        row3(U, v, U.i0 + nx, U.y < ny - 1, rn);
#pragma unroll
        for (int k = 0; k < V; ++k) {
            o[0][k] = rs[k];
            o[1][k] = rs[k + 1];
            o[2][k] = rs[k + 2];
            o[3][k] = rc[k];
            o[4][k] = rc[k + 1];
            o[5][k] = rc[k + 2];
            o[6][k] = rn[k];
            o[7][k] = rn[k + 1];
            o[8][k] = rn[k + 2];
        }
    }
    __device__ __forceinline__ int colour(const Unit &U, int k) const {
        return ((U.x0 + k) & 1) + 2 * (U.y & 1);
    }
    __device__ __forceinline__ void diag(const Unit &U, real (&d)[V]) const { vld<real, V>(C + U.i0, d); }
    __device__ __forceinline__ const real *diag_ptr() const { return C; }
    template <typename T>
    __device__ __forceinline__ void own(const Unit &U, const T *__restrict__ p, T (&o)[V]) const {
        vld<T, V>(p + U.i0, o);
    }
    template <typename T>
    __device__ __forceinline__ void put(const Unit &U, T *__restrict__ p, const T (&o)[V]) const {
        vst<T, V>(p + U.i0, o);
    }
};

template <typename real_, int V_>
struct U7 {
    using real = real_;
    static constexpr int V = V_, NB = 7, kC = 3;
    const real *C, *E, *N, *Up;
    int nx, ny, nz;
    int64_t n;
    struct Unit {
        int64_t i0;
        int x0, y, z;
        real a[NB][V];
    };
    __host__ __device__ int64_t units() const { return n / V; }
    __device__ __forceinline__ void geom(Unit &U, int64_t u) const {
        U.i0 = u * V;
        const int64_t pl = (int64_t)nx * ny;
        U.z = (int)((uint64_t)U.i0 / (uint64_t)pl);
        const int64_t r = U.i0 - (int64_t)U.z * pl;
        U.y = (int)((uint64_t)r / (uint64_t)nx);
        U.x0 = (int)(r - (int64_t)U.y * nx);
    }
    __device__ __forceinline__ void load(Unit &U, int64_t u) const {
        geom(U, u);
        const int64_t i0 = U.i0, pl = (int64_t)nx * ny;
        real c[V], e[V], nn[V], uu[V], ns[V], ud[V];
        vld<real, V>(C + i0, c);
        vld<real, V>(E + i0, e);
        vld<real, V>(N + i0, nn);
        vld<real, V>(Up + i0, uu);
        if (U.y > 0) vld<real, V>(N + i0 - nx, ns);
        else
#pragma unroll
            for (int k = 0; k < V; ++k) ns[k] = real(0);
        if (U.z > 0) vld<real, V>(Up + i0 - pl, ud);
        else
#pragma unroll
            for (int k = 0; k < V; ++k) ud[k] = real(0);
        const real ew = U.x0 > 0 ? E[i0 - 1] : real(0);
#pragma unroll
        for (int k = 0; k < V; ++k) {
            U.a[0][k] = ud[k];
            U.a[1][k] = ns[k];
            U.a[2][k] = k == 0 ? ew : e[k > 0 ? k - 1 : 0];
            U.a[3][k] = c[k];
            U.a[4][k] = e[k];
            U.a[5][k] = nn[k];
            U.a[6][k] = uu[k];
        }
    }
    __device__ __forceinline__ bool valid(const Unit &U, int s, int k) const {
        switch (s) {
        case 0: return U.z > 0;
        case 1: return U.y > 0;
        case 2: return U.x0 + k > 0;
        case 3: return true;
        case 4: return U.x0 + k < nx - 1;
        case 5: return U.y < ny - 1;
        default: return U.z < nz - 1;
        }
    }
    __device__ __forceinline__ bool is_diag(const Unit &, int s, int) const { return s == kC; }
    template <typename T>
    __device__ __forceinline__ void gather(const Unit &U, const T *__restrict__ v, T (&o)[NB][V]) const {
        const int64_t i0 = U.i0, pl = (int64_t)nx * ny;
        T c[V], d[V], sv[V], nv[V], uv[V];
        vld<T, V>(v + i0, c);
        if (U.z > 0) vld<T, V>(v + i0 - pl, d);
        else
#pragma unroll
            for (int k = 0; k < V; ++k) d[k] = T(0);
        if (U.y > 0) vld<T, V>(v + i0 - nx, sv);
        else
#pragma unroll
            for (int k = 0; k < V; ++k) sv[k] = T(0);
        if (U.y < ny - 1) vld<T, V>(v + i0 + nx, nv);
        else
#pragma unroll
            for (int k = 0; k < V; ++k) nv[k] = T(0);
        if (U.z < nz - 1) vld<T, V>(v + i0 + pl, uv);
        else
#pragma unroll
            for (int k = 0; k < V; ++k) uv[k] = T(0);
        const T w = U.x0 > 0 ? v[i0 - 1] : T(0);
        const T e = U.x0 + V < nx ? v[i0 + V] : T(0);
#pragma unroll
        for (int k = 0; k < V; ++k) {
            o[0][k] = d[k];
            o[1][k] = sv[k];
            o[2][k] = k == 0 ? w : c[k > 0 ? k - 1 : 0];
            o[3][k] = c[k];
            o[4][k] = k == V - 1 ? e : c[k < V - 1 ? k + 1 : 0];
            o[5][k] = nv[k];
            o[6][k] = uv[k];
        }
    }
    __device__ __forceinline__ int colour(const Unit &U, int k) const { return (U.x0 + k + U.y + U.z) & 1; }
    __device__ __forceinline__ void diag(const Unit &U, real (&d)[V]) const { vld<real, V>(C + U.i0, d); }
    __device__ __forceinline__ const real *diag_ptr() const { return C; }
    template <typename T>
    __device__ __forceinline__ void own(const Unit &U, const T *__restrict__ p, T (&o)[V]) const {
        vld<T, V>(p + U.i0, o);
    }
    template <typename T>
    __device__ __forceinline__ void put(const Unit &U, T *__restrict__ p, const T (&o)[V]) const {
        vst<T, V>(p + U.i0, o);
    }
};

// Restricted matrix B (K rows) in column-major ELL: slot s of row k at
// [s*K + k]; members in ascending column order, then col = -1 padding.
template <typename real_, int NB_>
struct UEll {
    using real = real_;
    static constexpr int V = 1, NB = NB_;
    const int32_t *col;
    const real *val;
    const real *dg;       // diagonal of B
    const uint8_t *clr;   // colour of each row (from the grid)
    int64_t n;            // K
    struct Unit {
        int64_t i0;
        int32_t c[NB];
        real a[NB][1];
    };
    __host__ __device__ int64_t units() const { return n; }
    __device__ __forceinline__ void geom(Unit &U, int64_t u) const { U.i0 = u; }
    __device__ __forceinline__ void load(Unit &U, int64_t u) const {
        U.i0 = u;
#pragma unroll
        for (int s = 0; s < NB; ++s) {
            U.c[s] = col[s * n + u];
            U.a[s][0] = val[s * n + u];
        }
    }
    __device__ __forceinline__ bool valid(const Unit &U, int s, int) const { return U.c[s] >= 0; }
    __device__ __forceinline__ bool is_diag(const Unit &U, int s, int) const { return U.c[s] == U.i0; }
    template <typename T>
    __device__ __forceinline__ void gather(const Unit &U, const T *__restrict__ v, T (&o)[NB][1]) const {
#pragma unroll
        for (int s = 0; s < NB; ++s) o[s][0] = U.c[s] >= 0 ? v[U.c[s]] : T(0);
    }
    __device__ __forceinline__ int colour(const Unit &U, int) const { return clr[U.i0]; }
    __device__ __forceinline__ void diag(const Unit &U, real (&d)[1]) const { d[0] = dg[U.i0]; }
    __device__ __forceinline__ const real *diag_ptr() const { return dg; }
    template <typename T>
    __device__ __forceinline__ void own(const Unit &U, const T *__restrict__ p, T (&o)[1]) const {
        o[0] = p[U.i0];
    }
    template <typename T>
    __device__ __forceinline__ void put(const Unit &U, T *__restrict__ p, const T (&o)[1]) const {
        p[U.i0] = o[0];
    }
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
