// Device-side building blocks of the local character-based solver (gfx950).
//
// Operators visit the stored entries of a row in ascending column order, so
// every per-row sum (residual, SpMV, gradient mimic, expansion bound,
// Gauss-Seidel update) has one fixed rounding sequence.  Reductions are
// deterministic: a fixed wave-shuffle / LDS tree per block writes one partial
// per block, and every block of the next kernel folds them in block order.
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
    // the same members with their stencil slots: S, W, C, E, N (ascending)
    static constexpr int kSlots = 5;
    template <class F>
    __device__ __forceinline__ void for_each_slot(int64_t i, F &&f) const {
        const int y = (int)((uint32_t)i / (uint32_t)nx);
        const int x = (int)i - y * nx;
        if (y > 0) f(0, i - nx, N[i - nx]);
        if (x > 0) f(1, i - 1, E[i - 1]);
        f(2, i, C[i]);
        if (x < nx - 1) f(3, i + 1, E[i]);
        if (y < ny - 1) f(4, i + nx, N[i]);
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
    // the same members with their stencil slots: SW, S, SE, W, C, E, NW, N,
    // NE (ascending)
    static constexpr int kSlots = 9;
    template <class F>
    __device__ __forceinline__ void for_each_slot(int64_t i, F &&f) const {
        const int y = (int)((uint32_t)i / (uint32_t)nx);
        const int x = (int)i - y * nx;
        const bool w = x > 0, e = x < nx - 1, s = y > 0, nn = y < ny - 1;
        if (s && w) f(0, i - nx - 1, NE[i - nx - 1]);
        if (s) f(1, i - nx, N[i - nx]);
        if (s && e) f(2, i - nx + 1, NW[i - nx + 1]);
        if (w) f(3, i - 1, E[i - 1]);
        f(4, i, C[i]);
        if (e) f(5, i + 1, E[i]);
        if (nn && w) f(6, i + nx - 1, NW[i]);
        if (nn) f(7, i + nx, N[i]);
        if (nn && e) f(8, i + nx + 1, NE[i]);
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
    // the same members with their stencil slots: D, S, W, C, E, N, U
    // (ascending)
    static constexpr int kSlots = 7;
    template <class F>
    __device__ __forceinline__ void for_each_slot(int64_t i, F &&f) const {
        const int64_t pl = (int64_t)nx * ny;
        const int z = (int)((uint64_t)i / (uint64_t)pl);
        const int r = (int)(i - (int64_t)z * pl);
        const int y = (int)((uint32_t)r / (uint32_t)nx);
        const int x = r - y * nx;
        if (z > 0) f(0, i - pl, U[i - pl]);
        if (y > 0) f(1, i - nx, N[i - nx]);
        if (x > 0) f(2, i - 1, E[i - 1]);
        f(3, i, C[i]);
        if (x < nx - 1) f(4, i + 1, E[i]);
        if (y < ny - 1) f(5, i + nx, N[i]);
        if (z < nz - 1) f(6, i + pl, U[i]);
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

// Nine-point operator in full storage (non-symmetric, e.g. with convection):
// a[s * n + i] is the coefficient of row i at slot s, slots in ascending
// column order SW, S, SE, W, C, E, NW, N, NE; entries whose neighbour lies
// outside the grid are ignored.
template <typename real>
struct Stencil9N {
    const real *a;
    int nx, ny;
    int64_t n;
    template <class F>
    __device__ __forceinline__ void for_each(int64_t i, F &&f) const {
        const int y = (int)((uint32_t)i / (uint32_t)nx);
        const int x = (int)i - y * nx;
        const bool w = x > 0, e = x < nx - 1, s = y > 0, nn = y < ny - 1;
        if (s && w) f(i - nx - 1, a[i]);
        if (s) f(i - nx, a[n + i]);
        if (s && e) f(i - nx + 1, a[2 * n + i]);
        if (w) f(i - 1, a[3 * n + i]);
        f(i, a[4 * n + i]);
        if (e) f(i + 1, a[5 * n + i]);
        if (nn && w) f(i + nx - 1, a[6 * n + i]);
        if (nn) f(i + nx, a[7 * n + i]);
        if (nn && e) f(i + nx + 1, a[8 * n + i]);
    }
    // the same members with their slots: SW, S, SE, W, C, E, NW, N, NE
    static constexpr int kSlots = 9;
    template <class F>
    __device__ __forceinline__ void for_each_slot(int64_t i, F &&f) const {
        const int y = (int)((uint32_t)i / (uint32_t)nx);
        const int x = (int)i - y * nx;
        const bool w = x > 0, e = x < nx - 1, s = y > 0, nn = y < ny - 1;
        if (s && w) f(0, i - nx - 1, a[i]);
        if (s) f(1, i - nx, a[n + i]);
        if (s && e) f(2, i - nx + 1, a[2 * n + i]);
        if (w) f(3, i - 1, a[3 * n + i]);
        f(4, i, a[4 * n + i]);
        if (e) f(5, i + 1, a[5 * n + i]);
        if (nn && w) f(6, i + nx - 1, a[6 * n + i]);
        if (nn) f(7, i + nx, a[7 * n + i]);
        if (nn && e) f(8, i + nx + 1, a[8 * n + i]);
    }
    __device__ __forceinline__ real diag(int64_t i) const { return a[4 * n + i]; }
    __device__ __forceinline__ int colour(int64_t i) const {
        const int y = (int)((uint32_t)i / (uint32_t)nx);
        return (((int)i - y * nx) & 1) + 2 * (y & 1);
    }
    static constexpr int kColours = 4;
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

// Non-temporal vector load: for arrays that a pass reads exactly once (the
// own-cell coefficients), so they do not displace the vectors that
// neighbouring strips read again.
template <typename T, int V>
__device__ __forceinline__ void vld_nt(const T *__restrict__ p, T (&o)[V]) {
    if constexpr (V == 1) {
        o[0] = __builtin_nontemporal_load(p);
    } else {
        typedef T vt __attribute__((ext_vector_type(V)));
        const vt t = __builtin_nontemporal_load(reinterpret_cast<const vt *>(p));
#pragma unroll
        for (int k = 0; k < V; ++k) o[k] = t[k];
    }
}
// The choice is a template parameter: a run-time flag lets the compiler merge
// the two loads and drop the hint.
template <bool kNT, typename T, int V>
__device__ __forceinline__ void vld_sel(const T *__restrict__ p, T (&o)[V]) {
    if constexpr (kNT) vld_nt<T, V>(p, o);
    else vld<T, V>(p, o);
}
template <bool kNT, typename T, int V>
__device__ __forceinline__ void vst_sel(T *__restrict__ p, const T (&o)[V]) {
    if constexpr (!kNT) {
        vst<T, V>(p, o);
    } else if constexpr (V == 1) {
        __builtin_nontemporal_store(o[0], p);
    } else {
        typedef T vt __attribute__((ext_vector_type(V)));
        vt t;
#pragma unroll
        for (int k = 0; k < V; ++k) t[k] = o[k];
        __builtin_nontemporal_store(t, reinterpret_cast<vt *>(p));
    }
}

// Three consecutive grid rows of one vector around a strip of V cells, with
// one halo cell on each side: r[0] = column x0-1, r[1..V] = x0..x0+V-1,
// r[V+1] = x0+V (zero outside the grid or when not asked for).
template <typename T, int V>
struct Rows {
    T s[V + 2], c[V + 2], n[V + 2];
};
template <typename T, int V>
__device__ __forceinline__ void row_load(const T *__restrict__ v, int64_t base, int64_t safe, int x0,
                                         int nx, bool on, bool halo, T (&r)[V + 2]) {
    // straight-line: the strip is loaded from base when the row exists, else
    // from the in-range row safe, and selected to zero
    const int64_t b = on ? base : safe;
    T m[V];
    vld<T, V>(v + b, m);
    const T w = (on && halo && x0 > 0) ? v[b - 1] : T(0);
    const T e = (on && halo && x0 + V < nx) ? v[b + V] : T(0);
    r[0] = w;
#pragma unroll
    for (int k = 0; k < V; ++k) r[k + 1] = on ? m[k] : T(0);
    r[V + 1] = e;
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

// Row marching.  A wave owns a tile: a strip of 64 units of one grid row
// (lane l -> unit l of the strip; 3-D: of one plane) over mh consecutive rows
// (3-D: planes), and walks up.  The coefficients of the row below (south faces) and the
// rows y-1, y of every gathered vector stay in registers from the previous
// step, so each row is fetched once per pass instead of three times.  The
// per-cell sums are the same FMA chains as in the flat walk.
// Walk mode W of a 2-D operator: 0 the flat band walk, 1 row marching, 2 row
// marching with non-temporal loads of the own-cell coefficient arrays and
// non-temporal stores (for passes that stream more than the last-level cache).
struct MarchGeom {
    int mh;    // rows per tile
};
__host__ __device__ inline int64_t march_strips(int64_t upr) { return (upr + kWave - 1) / kWave; }

template <typename real_, int V_, int W_>
struct U5 {
    using real = real_;
    static constexpr int V = V_, NB = 5, kC = 2;
    static constexpr bool kMarch = W_ > 0, kNT = W_ == 2;
    static constexpr bool kCenter = true;   // slot kC of a gather is the own cell
    const real *C, *E, *N;
    int nx, ny;
    int64_t n;
    MarchGeom mg;
    struct Unit {
        int64_t i0;
        int x0, y;
        real a[NB][V];
    };
    __host__ __device__ int64_t units() const { return n / V; }
    __host__ __device__ int64_t upr() const { return nx / V; }
    __host__ __device__ int rows() const { return ny; }
    __host__ __device__ int64_t tiles() const {
        return march_strips(upr()) * (int64_t)((ny + mg.mh - 1) / mg.mh);
    }
    // south faces of row y: N of row y-1
    struct South {
        real ns[V];
    };
    __device__ __forceinline__ void south_init(South &S, const Unit &U) const {
        const bool s = U.y > 0;
        real t[V];
        vld<real, V>(N + (s ? U.i0 - nx : U.i0), t);
#pragma unroll
        for (int k = 0; k < V; ++k) S.ns[k] = s ? t[k] : real(0);
    }
    __device__ __forceinline__ void load_row(Unit &U, South &S) const {
        const int64_t i0 = U.i0;
        real c[V], e[V], nn[V];
        vld_sel<kNT, real, V>(C + i0, c);
        vld_sel<kNT, real, V>(E + i0, e);
        vld<real, V>(N + i0, nn);
        real ex[V + 1];   // E at columns x0-1 .. x0+V-1
        ex[0] = U.x0 > 0 ? E[i0 - 1] : real(0);
#pragma unroll
        for (int k = 0; k < V; ++k) ex[k + 1] = e[k];
#pragma unroll
        for (int k = 0; k < V; ++k) {
            U.a[0][k] = S.ns[k];
            U.a[1][k] = ex[k];
            U.a[2][k] = c[k];
            U.a[3][k] = e[k];
            U.a[4][k] = nn[k];
            S.ns[k] = nn[k];
        }
    }
    template <typename T>
    __device__ __forceinline__ void rows_init(Rows<T, V> &R, const T *__restrict__ v, const Unit &U) const {
        row_load<T, V>(v, U.i0 - nx, U.i0, U.x0, nx, U.y > 0, false, R.s);
        row_load<T, V>(v, U.i0, U.i0, U.x0, nx, true, true, R.c);
    }
    template <typename T>
    __device__ __forceinline__ void rows_next(Rows<T, V> &R, const T *__restrict__ v, const Unit &U) const {
        row_load<T, V>(v, U.i0 + nx, U.i0, U.x0, nx, U.y < ny - 1, true, R.n);
    }
    template <typename T>
    __device__ __forceinline__ void rows_slots(const Rows<T, V> &R, T (&o)[NB][V]) const {
#pragma unroll
        for (int k = 0; k < V; ++k) {
            o[0][k] = R.s[k + 1];
            o[1][k] = R.c[k];
            o[2][k] = R.c[k + 1];
            o[3][k] = R.c[k + 2];
            o[4][k] = R.n[k + 1];
        }
    }
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
    __host__ __device__ __forceinline__ const real *diag_ptr() const { return C; }
    template <typename T>
    __device__ __forceinline__ void own(const Unit &U, const T *__restrict__ p, T (&o)[V]) const {
        vld<T, V>(p + U.i0, o);
    }
    template <typename T>
    __device__ __forceinline__ void put(const Unit &U, T *__restrict__ p, const T (&o)[V]) const {
        vst_sel<kNT, T, V>(p + U.i0, o);
    }
    // geometry of unit u, unit xu of grid row `row`, known to the row walk
    __device__ __forceinline__ void geom_walk(Unit &U, int64_t u, int xu, int row) const {
        U.i0 = u * V;
        U.x0 = xu * V;
        U.y = row;
    }
    // carried rows of a gathered vector and their shift to the next row
    template <typename T>
    using Carry = Rows<T, V>;
    template <typename T>
    __device__ __forceinline__ void rows_shift(Rows<T, V> &R) const {
#pragma unroll
        for (int k = 0; k < V + 2; ++k) {
            R.s[k] = R.c[k];
            R.c[k] = R.n[k];
        }
    }
};

template <typename real_, int V_, int W_>
struct U9 {
    using real = real_;
    static constexpr int V = V_, NB = 9, kC = 4;
    static constexpr bool kMarch = W_ > 0, kNT = W_ == 2;
    static constexpr bool kCenter = true;
    const real *C, *E, *N, *NE, *NW;
    int nx, ny;
    int64_t n;
    MarchGeom mg;
    struct Unit {
        int64_t i0;
        int x0, y;
        real a[NB][V];
    };
    __host__ __device__ int64_t units() const { return n / V; }
    __host__ __device__ int64_t upr() const { return nx / V; }
    __host__ __device__ int rows() const { return ny; }
    __host__ __device__ int64_t tiles() const {
        return march_strips(upr()) * (int64_t)((ny + mg.mh - 1) / mg.mh);
    }
    // south faces of row y, all from row y-1: ne[k] = NE at column x0+k-1,
    // n[k] = N at x0+k, nw[k] = NW at x0+k (k = 0..V)
    struct South {
        real ne[V + 1], n[V], nw[V + 1];
    };
    // straight-line on purpose (loads from row y when there is no row y-1,
    // then selected away): branch-wise stores would be merged through a
    // pointer phi that keeps the carried state out of registers
    __device__ __forceinline__ void south_init(South &S, const Unit &U) const {
        const bool s = U.y > 0;
        const int64_t bs = s ? U.i0 - nx : U.i0;
        real tn[V], tne[V], tnw[V];
        vld<real, V>(N + bs, tn);
        vld<real, V>(NE + bs, tne);
        vld<real, V>(NW + bs, tnw);
        const real ne_w = (s && U.x0 > 0) ? NE[bs - 1] : real(0);
        const real nw_e = (s && U.x0 + V < nx) ? NW[bs + V] : real(0);
        S.ne[0] = ne_w;
#pragma unroll
        for (int k = 0; k < V; ++k) {
            S.n[k] = s ? tn[k] : real(0);
            S.ne[k + 1] = s ? tne[k] : real(0);
            S.nw[k] = s ? tnw[k] : real(0);
        }
        S.nw[V] = nw_e;
    }
    __device__ __forceinline__ void load_row(Unit &U, South &S) const {
        const int64_t i0 = U.i0;
        const bool w = U.x0 > 0, e = U.x0 + V < nx;
        real c[V], ee[V], nn[V], ne[V], nw[V];
        vld_sel<kNT, real, V>(C + i0, c);
        vld_sel<kNT, real, V>(E + i0, ee);
        vld<real, V>(N + i0, nn);
        vld<real, V>(NE + i0, ne);
        vld<real, V>(NW + i0, nw);
        real ex[V + 1];   // E at columns x0-1 .. x0+V-1
        ex[0] = w ? E[i0 - 1] : real(0);
#pragma unroll
        for (int k = 0; k < V; ++k) ex[k + 1] = ee[k];
        const real ne_w = w ? NE[i0 - 1] : real(0);   // NE at x0-1 of this row
        const real nw_e = e ? NW[i0 + V] : real(0);   // NW at x0+V of this row
#pragma unroll
        for (int k = 0; k < V; ++k) {
            U.a[0][k] = S.ne[k];
            U.a[1][k] = S.n[k];
            U.a[2][k] = S.nw[k + 1];
            U.a[3][k] = ex[k];
            U.a[4][k] = c[k];
            U.a[5][k] = ee[k];
            U.a[6][k] = nw[k];
            U.a[7][k] = nn[k];
            U.a[8][k] = ne[k];
        }
        S.ne[0] = ne_w;
#pragma unroll
        for (int k = 0; k < V; ++k) {
            S.ne[k + 1] = ne[k];
            S.n[k] = nn[k];
            S.nw[k] = nw[k];
        }
        S.nw[V] = nw_e;
    }
    template <typename T>
    __device__ __forceinline__ void rows_init(Rows<T, V> &R, const T *__restrict__ v, const Unit &U) const {
        row_load<T, V>(v, U.i0 - nx, U.i0, U.x0, nx, U.y > 0, true, R.s);
        row_load<T, V>(v, U.i0, U.i0, U.x0, nx, true, true, R.c);
    }
    template <typename T>
    __device__ __forceinline__ void rows_next(Rows<T, V> &R, const T *__restrict__ v, const Unit &U) const {
        row_load<T, V>(v, U.i0 + nx, U.i0, U.x0, nx, U.y < ny - 1, true, R.n);
    }
    template <typename T>
    __device__ __forceinline__ void rows_slots(const Rows<T, V> &R, T (&o)[NB][V]) const {
#pragma unroll
        for (int k = 0; k < V; ++k) {
            o[0][k] = R.s[k];
            o[1][k] = R.s[k + 1];
            o[2][k] = R.s[k + 2];
            o[3][k] = R.c[k];
            o[4][k] = R.c[k + 1];
            o[5][k] = R.c[k + 2];
            o[6][k] = R.n[k];
            o[7][k] = R.n[k + 1];
            o[8][k] = R.n[k + 2];
        }
    }
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
    __host__ __device__ __forceinline__ const real *diag_ptr() const { return C; }
    template <typename T>
    __device__ __forceinline__ void own(const Unit &U, const T *__restrict__ p, T (&o)[V]) const {
        vld<T, V>(p + U.i0, o);
    }
    template <typename T>
    __device__ __forceinline__ void put(const Unit &U, T *__restrict__ p, const T (&o)[V]) const {
        vst_sel<kNT, T, V>(p + U.i0, o);
    }
    // geometry of unit u, unit xu of grid row `row`, known to the row walk
    __device__ __forceinline__ void geom_walk(Unit &U, int64_t u, int xu, int row) const {
        U.i0 = u * V;
        U.x0 = xu * V;
        U.y = row;
    }
    // carried rows of a gathered vector and their shift to the next row
    template <typename T>
    using Carry = Rows<T, V>;
    template <typename T>
    __device__ __forceinline__ void rows_shift(Rows<T, V> &R) const {
#pragma unroll
        for (int k = 0; k < V + 2; ++k) {
            R.s[k] = R.c[k];
            R.c[k] = R.n[k];
        }
    }
};

// Full-storage nine-point unit operator (Stencil9N's layout), flat walk only:
// every coefficient is the own row's, so a unit loads nine contiguous strips.
template <typename real_, int V_>
struct U9N {
    using real = real_;
    static constexpr int V = V_, NB = 9, kC = 4;
    static constexpr bool kMarch = false, kNT = false, kCenter = true;
    const real *a;   // [9][n]
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
#pragma unroll
        for (int s = 0; s < NB; ++s) vld<real, V>(a + s * n + U.i0, U.a[s]);
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
    __device__ __forceinline__ void diag(const Unit &U, real (&d)[V]) const {
        vld<real, V>(a + 4 * n + U.i0, d);
    }
    __host__ __device__ __forceinline__ const real *diag_ptr() const { return a + 4 * n; }
    template <typename T>
    __device__ __forceinline__ void own(const Unit &U, const T *__restrict__ p, T (&o)[V]) const {
        vld<T, V>(p + U.i0, o);
    }
    template <typename T>
    __device__ __forceinline__ void put(const Unit &U, T *__restrict__ p, const T (&o)[V]) const {
        vst<T, V>(p + U.i0, o);
    }
};

// operators whose matrix need not be symmetric (solved by GMRES), and the
// restricted ELL system (solved by GMRES when the full matrix is one of them)
template <class Op>
constexpr bool is_nonsym = false;
template <typename real, int V>
constexpr bool is_nonsym<U9N<real, V>> = true;
template <typename real, int NB>
struct UEll;
template <class Op>
constexpr bool is_ell = false;
template <typename real, int NB>
constexpr bool is_ell<UEll<real, NB>> = true;

template <typename real_, int V_, int W_>
struct U7 {
    using real = real_;
    static constexpr int V = V_, NB = 7, kC = 3;
    static constexpr bool kMarch = W_ > 0, kNT = W_ == 2, kCenter = true;
    const real *C, *E, *N, *Up;
    int nx, ny, nz;
    int64_t n;
    MarchGeom mg;
    struct Unit {
        int64_t i0;
        int x0, y, z;
        real a[NB][V];
    };
    __host__ __device__ int64_t units() const { return n / V; }
    // Marching goes up the planes: a tile is 64 strips of one plane (lanes
    // cover grid rows y of the plane) over mh planes.  Carried: the rows of
    // planes z-1, z at this (y) and the Up coefficients of plane z-1; the
    // in-plane neighbour rows y-1, y+1 are loaded at every step (they are the
    // own rows of the neighbouring lanes / wavefronts at the same step).
    __host__ __device__ int64_t upr() const { return (int64_t)nx * ny / V; }
    __host__ __device__ int rows() const { return nz; }
    __host__ __device__ int64_t tiles() const {
        return march_strips(upr()) * (int64_t)((nz + mg.mh - 1) / mg.mh);
    }
    __device__ __forceinline__ void geom_walk(Unit &U, int64_t u, int xu, int row) const {
        const int upx = nx / V;
        U.i0 = u * V;
        U.y = xu / upx;
        U.x0 = (xu - U.y * upx) * V;
        U.z = row;
    }
    struct South {
        real ud[V];   // Up of plane z-1 (the face below)
    };
    __device__ __forceinline__ void south_init(South &S, const Unit &U) const {
        const int64_t pl = (int64_t)nx * ny;
        const bool d = U.z > 0;
        real t[V];
        vld<real, V>(Up + (d ? U.i0 - pl : U.i0), t);
#pragma unroll
        for (int k = 0; k < V; ++k) S.ud[k] = d ? t[k] : real(0);
    }
    __device__ __forceinline__ void load_row(Unit &U, South &S) const {
        const int64_t i0 = U.i0;
        const bool s = U.y > 0;
        real c[V], e[V], nn[V], uu[V], ts[V];
        vld_sel<kNT, real, V>(C + i0, c);
        vld_sel<kNT, real, V>(E + i0, e);
        vld<real, V>(N + i0, nn);
        vld_sel<kNT, real, V>(Up + i0, uu);
        vld<real, V>(N + (s ? i0 - nx : i0), ts);
        real ex[V + 1];   // E at columns x0-1 .. x0+V-1
        ex[0] = U.x0 > 0 ? E[i0 - 1] : real(0);
#pragma unroll
        for (int k = 0; k < V; ++k) ex[k + 1] = e[k];
#pragma unroll
        for (int k = 0; k < V; ++k) {
            U.a[0][k] = S.ud[k];
            U.a[1][k] = s ? ts[k] : real(0);
            U.a[2][k] = ex[k];
            U.a[3][k] = c[k];
            U.a[4][k] = e[k];
            U.a[5][k] = nn[k];
            U.a[6][k] = uu[k];
            S.ud[k] = uu[k];
        }
    }
    template <typename T>
    struct Carry {
        T s[V + 2], c[V + 2], n[V + 2];   // planes z-1, z, z+1 at this (y)
        T ys[V], yn[V];                   // rows y-1, y+1 of plane z
    };
    template <typename T>
    __device__ __forceinline__ void rows_init(Carry<T> &R, const T *__restrict__ v, const Unit &U) const {
        const int64_t pl = (int64_t)nx * ny;
        row_load<T, V>(v, U.i0 - pl, U.i0, U.x0, nx, U.z > 0, false, R.s);
        row_load<T, V>(v, U.i0, U.i0, U.x0, nx, true, true, R.c);
    }
    template <typename T>
    __device__ __forceinline__ void rows_next(Carry<T> &R, const T *__restrict__ v, const Unit &U) const {
        const int64_t pl = (int64_t)nx * ny;
        row_load<T, V>(v, U.i0 + pl, U.i0, U.x0, nx, U.z < nz - 1, true, R.n);
        const bool s = U.y > 0, no = U.y < ny - 1;
        T a[V], b[V];
        vld<T, V>(v + (s ? U.i0 - nx : U.i0), a);
        vld<T, V>(v + (no ? U.i0 + nx : U.i0), b);
#pragma unroll
        for (int k = 0; k < V; ++k) {
            R.ys[k] = s ? a[k] : T(0);
            R.yn[k] = no ? b[k] : T(0);
        }
    }
    template <typename T>
    __device__ __forceinline__ void rows_slots(const Carry<T> &R, T (&o)[NB][V]) const {
#pragma unroll
        for (int k = 0; k < V; ++k) {
            o[0][k] = R.s[k + 1];
            o[1][k] = R.ys[k];
            o[2][k] = R.c[k];
            o[3][k] = R.c[k + 1];
            o[4][k] = R.c[k + 2];
            o[5][k] = R.yn[k];
            o[6][k] = R.n[k + 1];
        }
    }
    template <typename T>
    __device__ __forceinline__ void rows_shift(Carry<T> &R) const {
#pragma unroll
        for (int k = 0; k < V + 2; ++k) {
            R.s[k] = R.c[k];
            R.c[k] = R.n[k];
        }
    }
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
    __host__ __device__ __forceinline__ const real *diag_ptr() const { return C; }
    template <typename T>
    __device__ __forceinline__ void own(const Unit &U, const T *__restrict__ p, T (&o)[V]) const {
        vld<T, V>(p + U.i0, o);
    }
    template <typename T>
    __device__ __forceinline__ void put(const Unit &U, T *__restrict__ p, const T (&o)[V]) const {
        vst_sel<kNT, T, V>(p + U.i0, o);
    }
};

// Restricted matrix B (K rows) in column-major ELL: slot s of row k at
// [s*K + k]; members in ascending column order, then col = -1 padding.
template <typename real_, int NB_>
struct UEll {
    using real = real_;
    static constexpr int V = 1, NB = NB_;
    static constexpr bool kMarch = false;
    static constexpr bool kCenter = false;   // the diagonal slot varies by row
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
    __host__ __device__ __forceinline__ const real *diag_ptr() const { return dg; }
    template <typename T>
    __device__ __forceinline__ void own(const Unit &U, const T *__restrict__ p, T (&o)[1]) const {
        o[0] = p[U.i0];
    }
    template <typename T>
    __device__ __forceinline__ void put(const Unit &U, T *__restrict__ p, const T (&o)[1]) const {
        p[U.i0] = o[0];
    }
};

// B of a domain in grid order on the five- or nine-point stencil, with its
// columns coded per row instead of per member.  The values sit in the
// stencil's fixed slots (S, W, C, E, N or SW, S, SE, W, C, E, NW, N, NE:
// ascending column order, zero where the neighbour is outside the grid or
// the domain).  A member's column follows from the row's position k, a
// presence bit and, for the rows below and above, soff / noff = p - k (two
// 16-bit halves of one word), p being the number of domain cells before the
// cell straight below (above) in grid order: W = k - 1, E = k + 1, S = p,
// SW = p - 1, SE = p + [S present], and the same above.  5 bytes per row
// instead of 4 per member, for domains whose rows reach at most kMaxCol16
// rows away; the same members, order and arithmetic as UEll.
//
// Only the upper half of the slots is stored (C, E, N or C, E, NW, N, NE:
// slot s at val[(s - centre) * K + k]).  The stencils are stored as half
// stencils, so B is symmetric to the bit, and the coupling with a member j
// below or to the left is j's own entry in the mirrored slot (NB - 1 - s).
// Each row still loads NB values, but the lower ones come from rows that
// neighbouring lanes and waves load too.
constexpr int64_t kMaxCol16 = 32767;

struct RowCode {
    const uint32_t *off;   // (uint16) soff | (uint16) noff << 16
    const uint8_t *mask;   // bit b: slot b (b < centre) or b + 1 present
};

template <typename real_, int NB_>
struct UEllShort : UEll<real_, NB_> {
    static_assert(NB_ == 5 || NB_ == 9, "row codes of the 2-D stencils");
    using Base = UEll<real_, NB_>;
    using Unit = typename Base::Unit;
    static constexpr int kMid = NB_ / 2;
    RowCode code;
    __device__ __forceinline__ void load(Unit &U, int64_t u) const {
        U.i0 = u;
        const int k = (int)u;
        const uint32_t w = code.off[u];
        const int so = k + (int)(int16_t)(w & 0xffffu), no = k + (int)(int16_t)(w >> 16);
        const unsigned m = code.mask[u];
        auto has = [&](int sl) -> int { return (int)((m >> (sl < kMid ? sl : sl - 1)) & 1u); };
        if constexpr (NB_ == 9) {
            U.c[0] = has(0) ? so - 1 : -1;
            U.c[1] = has(1) ? so : -1;
            U.c[2] = has(2) ? so + has(1) : -1;
            U.c[3] = has(3) ? k - 1 : -1;
            U.c[4] = k;
            U.c[5] = has(5) ? k + 1 : -1;
            U.c[6] = has(6) ? no - 1 : -1;
            U.c[7] = has(7) ? no : -1;
            U.c[8] = has(8) ? no + has(7) : -1;
        } else {
            U.c[0] = has(0) ? so : -1;
            U.c[1] = has(1) ? k - 1 : -1;
            U.c[2] = k;
            U.c[3] = has(3) ? k + 1 : -1;
            U.c[4] = has(4) ? no : -1;
        }
#pragma unroll
        for (int sl = kMid; sl < NB_; ++sl) U.a[sl][0] = this->val[(sl - kMid) * this->n + u];
        // the lower slots from the members' mirrored entries; an absent
        // member (c = -1) reads the last entry of the slot before, in bounds,
        // and is masked
#pragma unroll
        for (int sl = 0; sl < kMid; ++sl) {
            const int j = U.c[sl];
            const real_ t = this->val[(NB_ - 1 - sl - kMid) * this->n + j];
            U.a[sl][0] = j >= 0 ? t : real_(0);
        }
    }
};
template <typename real, int NB>
constexpr bool is_ell<UEllShort<real, NB>> = true;

// B of a red-black colour-blocked domain (two colours, rows colour by
// colour, each colour in grid order) on the five- or seven-point stencil,
// coded per row.  The values sit in the stencil's fixed slots (S, W, C, E, N
// or D, S, W, C, E, N, U: grid order, as in the blocked UEll rows).  Every
// neighbour has the other colour, so a row keeps q, the position the other
// colour's block gives a cell at the row's own grid index (the number of
// its members before it, plus the block's start), and unsigned 16-bit
// distances (one 64-bit word) to the members straight below and above:
// W = q - 1, E = q, S = q - ds, N = q + dn, D = q - dd, U = q + du.  9 or 13
// bytes per row instead of 4 per member; the same members, order and
// arithmetic as UEll.  A distance counts members of the other colour in
// half a row or half a plane: at most 65535 while that reach is at most
// kMaxRB16 cells.
constexpr int64_t kMaxRB16 = 131068;

struct RBCode {
    const uint64_t *d;     // ds | dn << 16 | dd << 32 | du << 48 (dd, du: seven-point only)
    const int32_t *q;
    const uint8_t *mask;   // bit b: slot b (b < centre) or b + 1 present
};

template <typename real_, int NB_>
struct UEllRB : UEll<real_, NB_> {
    static_assert(NB_ == 5 || NB_ == 7, "red-black row codes of the five- and seven-point stencils");
    using Base = UEll<real_, NB_>;
    using Unit = typename Base::Unit;
    static constexpr int kMid = NB_ / 2;
    RBCode code;
    __device__ __forceinline__ void load(Unit &U, int64_t u) const {
        U.i0 = u;
        const uint64_t w = code.d[u];
        const int q = code.q[u];
        const unsigned m = code.mask[u];
        const int ds = (int)(w & 0xffffu), dn = (int)((w >> 16) & 0xffffu);
        auto has = [&](int sl) -> bool { return (m >> (sl < kMid ? sl : sl - 1)) & 1u; };
        if constexpr (NB_ == 7) {
            const int dd = (int)((w >> 32) & 0xffffu), du = (int)(w >> 48);
            U.c[0] = has(0) ? q - dd : -1;
            U.c[1] = has(1) ? q - ds : -1;
            U.c[2] = has(2) ? q - 1 : -1;
            U.c[3] = (int)u;
            U.c[4] = has(4) ? q : -1;
            U.c[5] = has(5) ? q + dn : -1;
            U.c[6] = has(6) ? q + du : -1;
        } else {
            U.c[0] = has(0) ? q - ds : -1;
            U.c[1] = has(1) ? q - 1 : -1;
            U.c[2] = (int)u;
            U.c[3] = has(3) ? q : -1;
            U.c[4] = has(4) ? q + dn : -1;
        }
#pragma unroll
        for (int sl = 0; sl < NB_; ++sl) U.a[sl][0] = this->val[sl * this->n + u];
    }
};
template <typename real, int NB>
constexpr bool is_ell<UEllRB<real, NB>> = true;


// ---------------------------------------------------------------------------
// walks: the order in which a grid-sized kernel visits its units
// ---------------------------------------------------------------------------
// Kernel loop:  for (auto W = walk<NG>(A); W.valid(); W.advance()) {
//                   W.load(U);  W.template gather<j>(U, v_j, o);  ... }
// NG is the number of gathered vectors; gather<j> must be called for the same
// vector at every unit of a launch, and load() at every unit or at none.
template <class Op, int NG>
struct FlatWalk {
    using Unit = typename Op::Unit;
    Band B;
    __device__ __forceinline__ explicit FlatWalk(const Op &a) : B(my_band(a.units())) {}
    __device__ __forceinline__ bool valid() const { return B.u < B.end; }
    __device__ __forceinline__ void geom(const Op &A, Unit &U) const { A.geom(U, B.u); }
    __device__ __forceinline__ void load(const Op &A, Unit &U) { A.load(U, B.u); }
    template <int j>
    __device__ __forceinline__ void gather(const Op &A, const Unit &U, const typename Op::real *__restrict__ v,
                                           typename Op::real (&o)[Op::NB][Op::V]) {
        A.gather(U, v, o);
    }
    __device__ __forceinline__ void advance() { B.u += B.step; }
};

template <class Op, int NG>
struct RowWalk {
    using real = typename Op::real;
    using Unit = typename Op::Unit;
    static constexpr int V = Op::V;
    int64_t u, upr, t, tiles, strips;
    int left, mh, nrows, row, xu;
    int fresh;
    typename Op::South S;
    typename Op::template Carry<real> R[NG > 0 ? NG : 1];
    __device__ __forceinline__ explicit RowWalk(const Op &a) {
        upr = a.upr();
        strips = march_strips(upr);
        tiles = a.tiles();
        mh = a.mg.mh;
        nrows = a.rows();
        t = (int64_t)logical_block() * kWaves + threadIdx.x / kWave;
        start();
    }
    __device__ __forceinline__ void start() {
        const int lane = threadIdx.x % kWave;
        left = 0;
        for (; t < tiles; t += (int64_t)gridDim.x * kWaves) {
            const int64_t strip = t % strips, seg = t / strips;
            const int64_t x = strip * kWave + lane;
            if (x >= upr) continue;
            row = (int)seg * mh;
            xu = (int)x;
            left = min(mh, nrows - row);
            u = (int64_t)row * upr + x;
            fresh = 1;
            return;
        }
    }
    __device__ __forceinline__ bool valid() const { return left > 0; }
    __device__ __forceinline__ void geom(const Op &A, Unit &U) const { A.geom_walk(U, u, xu, row); }
    __device__ __forceinline__ void load(const Op &A, Unit &U) {
        A.geom_walk(U, u, xu, row);
        if (fresh) A.south_init(S, U);
        A.load_row(U, S);
    }
    template <int j>
    __device__ __forceinline__ void gather(const Op &A, const Unit &U, const real *__restrict__ v,
                                           real (&o)[Op::NB][Op::V]) {
        static_assert(j < NG, "gather stream index out of range");
        auto &r = R[j];
        if (fresh) A.rows_init(r, v, U);
        A.rows_next(r, v, U);
        A.rows_slots(r, o);
        A.rows_shift(r);
    }
    __device__ __forceinline__ void advance() {
        fresh = 0;
        u += upr;
        ++row;
        if (--left == 0) {
            t += (int64_t)gridDim.x * kWaves;
            start();
        }
    }
};

template <int NG, class Op>
__device__ __forceinline__ auto walk(const Op &A) {
    if constexpr (Op::kMarch) return RowWalk<Op, NG>(A);
    else return FlatWalk<Op, NG>(A);
}

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
// gets bit-identical totals, valid in all of its threads.  A thread issues
// the loads of kFoldLoads strided partials of every value before it combines
// any of them, so a fold over g <= kFoldLoads x kBlock partials waits for one
// round of cache latency rather than g / kBlock rounds in sequence (this fold
// opens every launch of the iterative kernels).
constexpr int kFoldLoads = 4;
template <typename T, int NV, class O>
__device__ __forceinline__ void read_partials(const T *part, int g, O ops, T (&tot)[NV]) {
    __shared__ T lds[kWaves][NV];
    T a[NV];
#pragma unroll
    for (int k = 0; k < NV; ++k) a[k] = T(0);
    for (int b0 = threadIdx.x; b0 < g; b0 += kFoldLoads * kBlock) {
        T p[NV][kFoldLoads];
#pragma unroll
        for (int k = 0; k < NV; ++k)
#pragma unroll
            for (int m = 0; m < kFoldLoads; ++m) {
                const int b = b0 + m * kBlock;
                p[k][m] = b < g ? part[(size_t)k * g + b] : T(0);
            }
#pragma unroll
        for (int k = 0; k < NV; ++k)
#pragma unroll
            for (int m = 0; m < kFoldLoads; ++m) {
                const int b = b0 + m * kBlock;
                if (b < g) a[k] = (b == (int)threadIdx.x) ? p[k][m] : ops.template apply<T>(k, a[k], p[k][m]);
            }
    }
#pragma unroll
    for (int k = 0; k < NV; ++k)
        a[k] = ops.template reduce_wave<T>(k, a[k]);   // xor butterfly: the same in every lane
    const int w = threadIdx.x / kWave;
    if ((threadIdx.x & (kWave - 1)) == 0) {
#pragma unroll
        for (int k = 0; k < NV; ++k) lds[w][k] = a[k];
    }
    __syncthreads();
    // every thread combines the wave sums in the same order
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        T s = lds[0][k];
#pragma unroll
        for (int q = 1; q < kWaves; ++q) s = ops.template apply<T>(k, s, lds[q][k]);
        tot[k] = s;
    }
    __syncthreads();   // lds may be reused by the next fold
}

// exclusive prefix of integer block counts: sum of cnt[0..upto) in every
// thread, plus the grand total of cnt[0..g)
__device__ __forceinline__ void block_prefix_of_counts(const int32_t *cnt, int g, int upto,
                                                       int &before, int &total) {
    __shared__ int red[2][kWaves];
    int a = 0, t = 0;
    for (int b0 = threadIdx.x; b0 < g; b0 += kFoldLoads * kBlock) {
        int c[kFoldLoads];   // loads in flight together, as in read_partials
#pragma unroll
        for (int m = 0; m < kFoldLoads; ++m) c[m] = b0 + m * kBlock < g ? cnt[b0 + m * kBlock] : 0;
#pragma unroll
        for (int m = 0; m < kFoldLoads; ++m) {
            t += c[m];
            if (b0 + m * kBlock < upto) a += c[m];
        }
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
