// HIP kernels of the local character-based solver (gfx950, wave64).
//
// Per-row kernels use a chunked grid: block b (after the XCD remap) owns rows
// [b*chunk, (b+1)*chunk) and walks them 256 at a time, so loads are
// coalesced and stencil neighbours stay in the owning XCD's L2.  Kernels
// that reduce write per-block partials; the next kernel on the stream folds
// them in a fixed order at its start, so a solve is a stream of launches
// with no host round trip per iteration and no in-kernel cross-block fence.
#pragma once

#include "lcs_device.h"

namespace lcs {

// ---------------------------------------------------------------------------
// device state
// ---------------------------------------------------------------------------
// Every field is written by block 0 of one kernel and read only by later
// kernels on the stream (or by the host), never by other blocks of the kernel
// that writes it.
struct MarkState {
    double tau;       // threshold in use
    double smax;      // max |s_i|
    double bb;        // ||b||^2 (fixed-order block tree)
    int64_t K;        // |Omega| after compaction
    int32_t stop;     // an expansion round added nothing: later rounds are no-ops
    int32_t grown;    // rounds that added points
    double rr0;       // ||b - A x0||^2
    int32_t conv0;    // x0 already met the criterion: nothing was marked
    int32_t pad;
};

struct PcgState {
    double tol;       // absolute tolerance on the recursive ||r||
    double rz_next;   // r_j.z_j, formed by the A p kernel of iteration j
    double rz_cur;    // the r.z that the update of the previous iteration used
    double rr;        // ||r||^2 at exit
    double rr0;       // ||r_0||^2
    int32_t done, status, it, pad;
};

struct ResState {
    double rr, rmax, tol;
    int32_t done, status;
};

enum : int32_t { kStOk = 0, kStNoConv = 4, kStBreakdown = 5, kStNonFinite = 6 };

struct Scalars {
    MarkState ms;
    PcgState pcg;
    ResState res;
    double bnorm;        // ||b||_2
    double scale;        // refinement step scale max|r| (mixed precision)
    int64_t gather_nnz;  // nnz of the restricted matrix
    int32_t bad_idx;     // a caller-supplied domain was out of range or not ascending
    int32_t pad;
    int32_t saved_it[2];      // PCG iterations of the last global (0) / local (1) solve
    int32_t saved_status[2];
    double cg_gamma[2];       // single-synchronisation PCG: r_j.z_j by iteration parity
    double cg_alpha[2];       //                             alpha_j by iteration parity
    double scratch_norm;      // result of lcs_norm2_diff
    int64_t cstart[9];        // colour-blocked domain: first position of each colour, then K
};

// Own value of a gathered vector and the diagonal: for the stencils the
// gather's centre slot and the loaded C coefficients already hold them; the
// restricted matrix loads them.
template <class Op, typename T>
__device__ __forceinline__ void own_of(const Op &A, const typename Op::Unit &U,
                                       const T (&g)[Op::NB][Op::V], const T *__restrict__ v,
                                       T (&o)[Op::V]) {
    if constexpr (Op::kCenter) {
#pragma unroll
        for (int k = 0; k < Op::V; ++k) o[k] = g[Op::kC][k];
    } else {
        A.own(U, v, o);
    }
}
template <class Op>
__device__ __forceinline__ void diag_of(const Op &A, const typename Op::Unit &U,
                                        typename Op::real (&d)[Op::V]) {
    if constexpr (Op::kCenter) {
#pragma unroll
        for (int k = 0; k < Op::V; ++k) d[k] = U.a[Op::kC][k];
    } else {
        A.diag(U, d);
    }
}

// partial-sum slots (each kMaxGrid x 4 doubles: up to four values for each of
// up to 1024 blocks, or one value for each of up to 4096)
enum PartSlot { kPtScore = 0, kPtExp0, kPtExp1, kPtNorm, kPtRes, kPtAp, kPtUpd, kPtSgs, kPtSlots };
constexpr size_t kSlotElems = (size_t)kMaxGrid * 4;

// ---------------------------------------------------------------------------
// scores of Algorithms 2 and 3
// ---------------------------------------------------------------------------
// Residual mode: s = r^(0) = b - A x0 (FMA chain, ascending columns).
// Gradient mode: s = g, g_i = sum_{j != i} |x_i - x_j| (eq. grad).
// Partials: max |s_i|, ||b||^2 and ||r^(0)||^2 (the gradient mode forms r^(0)
// in registers for the last one).  xc (optional): a copy of x0, written from
// the values the pass has loaded anyway.
template <class Op, int kMode>
__global__ __launch_bounds__(kBlock) void k_score(Op A, const double *__restrict__ b,
                                                  const double *__restrict__ x,
                                                  double *__restrict__ s, double *part,
                                                  double *__restrict__ xc) {
    constexpr int V = Op::V, NB = Op::NB;
    double v[3] = {0.0, 0.0, 0.0};
    for (auto W = walk<1>(A); W.valid(); W.advance()) {
        typename Op::Unit U;
        W.load(A, U);
        double xv[NB][V], out[V], res[V], bb[V];
        W.template gather<0>(A, U, x, xv);
        A.own(U, b, bb);
#pragma unroll
        for (int k = 0; k < V; ++k) {
            double acc = bb[k];
#pragma unroll
            for (int q = 0; q < NB; ++q)
                if (A.valid(U, q, k)) acc = fma(-U.a[q][k], xv[q][k], acc);
            res[k] = acc;
            v[1] += bb[k] * bb[k];
            v[2] += acc * acc;
        }
        if (kMode == 0) {
#pragma unroll
            for (int k = 0; k < V; ++k) out[k] = res[k];
        } else {
            double xo[V];
            own_of(A, U, xv, x, xo);
#pragma unroll
            for (int k = 0; k < V; ++k) {
                double acc = 0.0;
#pragma unroll
                for (int q = 0; q < NB; ++q)
                    if (A.valid(U, q, k) && !A.is_diag(U, q, k)) acc += fabs(xo[k] - xv[q][k]);
                out[k] = acc;
            }
        }
        A.put(U, s, out);
        if (xc) {
            double xo[V];
            own_of(A, U, xv, x, xo);
            A.put(U, xc, xo);
        }
#pragma unroll
        for (int k = 0; k < V; ++k) {
            const double m = fabs(out[k]);
            v[0] = m > v[0] ? m : v[0];
        }
    }
    write_partials<double, 3>(v, Ops<1u>(), part);
}

// tau from the score partials: REL_MAX theta*max|s|, ABS theta,
// PAPER theta*||b||_2/sqrt(N); then stamp_i = (|s_i| > tau) (strict), zero on
// the padding [n, npad).  With eps0 >= 0, ||b|| from the score partials goes
// to sc->bnorm, and an x0 that already meets the criterion
// ||r^(0)|| <= eps0 ||b|| marks nothing and sets conv0.
__global__ __launch_bounds__(kBlock) void k_mark(const double *__restrict__ s,
                                                 uint8_t *__restrict__ stamp, int64_t n,
                                                 int64_t npad, int thresh, double theta,
                                                 double eps0, const double *part, int gprod,
                                                 Scalars *sc) {
    double tot[3];
    read_partials<double, 3>(part, gprod, Ops<1u>(), tot);
    double tau;
    if (thresh == 0) tau = theta * tot[0];
    else if (thresh == 1) tau = theta;
    else tau = theta * sqrt(tot[1]) / sqrt((double)n);
    const double bn = sqrt(tot[1]);
    const bool conv0 = eps0 >= 0.0 && sqrt(tot[2]) <= eps0 * bn;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        if (eps0 >= 0.0) sc->bnorm = bn;
        sc->ms.tau = tau;
        sc->ms.smax = tot[0];
        sc->ms.bb = tot[1];
        sc->ms.rr0 = tot[2];
        sc->ms.conv0 = conv0 ? 1 : 0;
        sc->ms.stop = 0;
        sc->ms.grown = 0;
    }
    // A block handles 2048 stamps per step (npad is a multiple of that
    // tile): the scores are read coalesced, eight per thread 256 apart, the
    // stamp bytes go through LDS, and each thread writes eight consecutive
    // stamps as one 64-bit word.
    __shared__ uint64_t tw[kBlock];
    uint8_t *tile = reinterpret_cast<uint8_t *>(tw);
    uint64_t *w = reinterpret_cast<uint64_t *>(stamp);
    for (int64_t base = (int64_t)blockIdx.x * kBlock * 8; base < npad;
         base += (int64_t)gridDim.x * kBlock * 8) {
        double v[8];
#pragma unroll
        for (int m = 0; m < 8; ++m) {
            const int64_t i = base + m * kBlock + threadIdx.x;
            v[m] = i < n ? s[i] : 0.0;
        }
#pragma unroll
        for (int m = 0; m < 8; ++m) {
            const int64_t i = base + m * kBlock + threadIdx.x;
            tile[m * kBlock + threadIdx.x] = (!conv0 && i < n && fabs(v[m]) > tau) ? 1 : 0;
        }
        __syncthreads();
        w[base / 8 + threadIdx.x] = tw[threadIdx.x];
        __syncthreads();
    }
}

// One synchronous expansion round m (Algorithm 3, eq. extend-local-condition):
// j outside Omega with a stored neighbour l in Omega (stamp 1..m) joins if
// |r_j| + sum_{l in Omega, ascending} |a_jl x_l| > tau.  New members get
// stamp m+1, which this round's readers treat as "outside".  Round m first
// reads round m-1's count: if it added nothing, this and later rounds are
// no-ops (Omega unchanged).
template <class Op>
__global__ __launch_bounds__(kBlock) void k_expand(Op A, const double *__restrict__ r,
                                                   const double *__restrict__ x,
                                                   uint8_t *stamp, int m, int64_t chunk,
                                                   const double *part_prev, double *part,
                                                   Scalars *sc) {
    if (sc->ms.stop) return;
    if (m >= 2) {
        double added[1];
        read_partials<double, 1>(part_prev, gridDim.x, Ops<0u>(), added);
        if (added[0] == 0.0) {
            if (blockIdx.x == 0 && threadIdx.x == 0) sc->ms.stop = 1;
            return;
        }
        if (blockIdx.x == 0 && threadIdx.x == 0) sc->ms.grown = m - 1;
    }
    const Chunk c = my_chunk(A.n, chunk);
    const double tau = sc->ms.tau;
    double v[1] = {0.0};
    for (int64_t j = c.begin + threadIdx.x; j < c.end; j += kBlock) {
        if (stamp[j] != 0) continue;
        // first the neighbours' stamps alone (the coefficient loads of this
        // visit are dead and dropped), so that rows away from Omega read no
        // coefficients
        bool nb = false;
        A.for_each(j, [&](int64_t l, double) {
            const int sl = stamp[l];
            if (l != j && sl != 0 && sl <= m) nb = true;
        });
        if (!nb) continue;
        double acc = fabs(r[j]);
        A.for_each(j, [&](int64_t l, double a) {
            const int sl = stamp[l];
            if (l != j && sl != 0 && sl <= m) acc += fabs(a * x[l]);
        });
        if (acc > tau) {
            stamp[j] = (uint8_t)(m + 1);
            v[0] += 1.0;
        }
    }
    write_partials<double, 1>(v, Ops<0u>(), part);
}

// The same round on a structured grid whose rows are a multiple of 8 cells:
// a thread takes eight cells at a time as one 64-bit word of stamps and
// reads the neighbouring rows' words, the bytes just left and right of its
// own, and on nine points the corners beside the rows below and above.  A
// word none of whose neighbours is stamped leaves at once; a cell with no
// neighbour in Omega costs a few byte tests and no scattered load.  Cells
// that do touch Omega take k_expand's test (same sum, same order), so the
// stamps are the same bit for bit.  kShape: 5 (2-D cross), 9 (2-D 3 x 3)
// or 7 (3-D cross, plane = nx * ny).
template <class Op, int kShape>
__global__ __launch_bounds__(kBlock) void k_expand_w(Op A, const double *__restrict__ r,
                                                     const double *__restrict__ x,
                                                     uint8_t *stamp, int m, int nx, int64_t plane,
                                                     const double *part_prev, double *part,
                                                     Scalars *sc) {
    if (sc->ms.stop) return;
    if (m >= 2) {
        double added[1];
        read_partials<double, 1>(part_prev, gridDim.x, Ops<0u>(), added);
        if (added[0] == 0.0) {
            if (blockIdx.x == 0 && threadIdx.x == 0) sc->ms.stop = 1;
            return;
        }
        if (blockIdx.x == 0 && threadIdx.x == 0) sc->ms.grown = m - 1;
    }
    const int64_t n = A.n, nw = n / 8, rw = nx / 8;
    const Chunk c = my_chunk(nw, (nw + gridDim.x - 1) / gridDim.x);
    const double tau = sc->ms.tau;
    const uint64_t *w = reinterpret_cast<const uint64_t *>(stamp);
    auto in = [&](int b) { return b != 0 && b <= m; };
    // grid positions by 32-bit division while the grid has < 2^32 cells
    const bool small = n <= (int64_t)0xffffffffu;
    auto div = [&](int64_t a, int64_t d) -> int64_t {
        return small ? (int64_t)((uint32_t)a / (uint32_t)d) : a / d;
    };
    // a row's eight stamps from its word, with the bytes e0 (x0 - 1) and e1
    // (x0 + 8) beside them
    auto unpack = [&](uint64_t v, int e0, int e1, int (&t)[10]) {
#pragma unroll
        for (int k = 0; k < 8; ++k) t[k + 1] = (int)((v >> (8 * k)) & 0xff);
        t[0] = e0;
        t[9] = e1;
    };
    double v[1] = {0.0};
    for (int64_t q = c.begin + threadIdx.x; q < c.end; q += kBlock) {
        const uint64_t own = w[q];
        // any cell outside Omega (a zero byte)?
        const uint64_t t = own | (own >> 4);
        const uint64_t t2 = t | (t >> 2);
        if ((((t2 | (t2 >> 1)) & 0x0101010101010101ull)) == 0x0101010101010101ull) continue;
        const int64_t i0 = q * 8;
        const int64_t rowi = div(i0, nx);
        const int x0 = (int)(i0 - rowi * nx);
        bool has_s, has_n, has_d = false, has_u = false;
        if (kShape == 7) {
            const int64_t z = div(i0, plane);
            const int y = (int)div(i0 - z * plane, nx);
            has_s = y > 0;
            has_n = (int64_t)(y + 1) * nx < plane;
            has_d = z > 0;
            has_u = (z + 1) * plane < n;
        } else {
            has_s = rowi > 0;
            has_n = i0 + nx < n;
        }
        const bool left = x0 > 0, right = x0 + 8 < nx;
        const uint64_t ws = has_s ? w[q - rw] : 0, wn = has_n ? w[q + rw] : 0;
        const uint64_t wd = has_d ? w[q - plane / 8] : 0, wu = has_u ? w[q + plane / 8] : 0;
        const int e0 = left ? stamp[i0 - 1] : 0, e1 = right ? stamp[i0 + 8] : 0;
        // the corners beside the rows below and above (nine points only)
        int s0 = 0, s1 = 0, n0 = 0, n1 = 0;
        if (kShape == 9) {
            s0 = has_s && left ? stamp[i0 - nx - 1] : 0;
            s1 = has_s && right ? stamp[i0 - nx + 8] : 0;
            n0 = has_n && left ? stamp[i0 + nx - 1] : 0;
            n1 = has_n && right ? stamp[i0 + nx + 8] : 0;
        }
        // no stamped cell among the neighbours: nothing can join
        if ((own | ws | wn | wd | wu) == 0 && (e0 | e1 | s0 | s1 | n0 | n1) == 0) continue;
        int cc[10], sn[10], nn[10], dn[10], up[10];
        unpack(own, e0, e1, cc);
        unpack(ws, s0, s1, sn);
        unpack(wn, n0, n1, nn);
        unpack(wd, 0, 0, dn);
        unpack(wu, 0, 0, up);
        // the neighbours' stamps come from these registers, not from memory:
        // during the round a stamp only changes from 0 to m + 1, and both
        // read as outside
        auto nstamp = [&](int sl, int k) -> int {
            if (kShape == 9) {
                switch (sl) {
                case 0: return sn[k - 1];
                case 1: return sn[k];
                case 2: return sn[k + 1];
                case 3: return cc[k - 1];
                case 5: return cc[k + 1];
                case 6: return nn[k - 1];
                case 7: return nn[k];
                case 8: return nn[k + 1];
                default: return 0;
                }
            } else if (kShape == 5) {
                switch (sl) {
                case 0: return sn[k];
                case 1: return cc[k - 1];
                case 3: return cc[k + 1];
                case 4: return nn[k];
                default: return 0;
                }
            } else {
                switch (sl) {
                case 0: return dn[k];
                case 1: return sn[k];
                case 2: return cc[k - 1];
                case 4: return cc[k + 1];
                case 5: return nn[k];
                case 6: return up[k];
                default: return 0;
                }
            }
        };
        uint64_t joined = 0;
#pragma unroll
        for (int k = 1; k <= 8; ++k) {
            if (cc[k] != 0) continue;
            bool nb = in(cc[k - 1]) || in(cc[k + 1]);
            if (has_s) nb = nb || in(sn[k]) || (kShape == 9 && (in(sn[k - 1]) || in(sn[k + 1])));
            if (has_n) nb = nb || in(nn[k]) || (kShape == 9 && (in(nn[k - 1]) || in(nn[k + 1])));
            if (has_d) nb = nb || in(dn[k]);
            if (has_u) nb = nb || in(up[k]);
            if (!nb) continue;
            const int64_t j = i0 + k - 1;
            double acc = fabs(r[j]);
            // the members in ascending order, the centre excluded (its
            // register stamp reads 0)
            A.for_each_slot(j, [&](int sl, int64_t l, double a) {
                if (in(nstamp(sl, k))) acc += fabs(a * x[l]);
            });
            if (acc > tau) {
                joined |= (uint64_t)(m + 1) << (8 * (k - 1));
                v[0] += 1.0;
            }
        }
        // the word's new members in one store (the word is this thread's)
        if (joined) reinterpret_cast<uint64_t *>(stamp)[q] = own | joined;
    }
    write_partials<double, 1>(v, Ops<0u>(), part);
}

// ---------------------------------------------------------------------------
// stream compaction: stamps -> idx (ascending), inv, K
// ---------------------------------------------------------------------------
// Tiles of 2048 stamps; thread t of a tile owns bytes [8t, 8t+8) read as one
// 64-bit word.
constexpr int kTile = kBlock * 8;

__device__ __forceinline__ int nonzero_bytes(uint64_t w) {
    uint64_t t = w | (w >> 4);
    t |= t >> 2;
    t |= t >> 1;
    t &= 0x0101010101010101ull;
    return __popcll(t);
}

// exclusive block scan of one int per thread; returns the prefix and the total
__device__ __forceinline__ int block_exclusive_scan(int v, int &total) {
    __shared__ int wsum[kWaves];
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    int inc = v;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        const int t = __shfl_up(inc, o, kWave);
        if (lane >= o) inc += t;
    }
    if (lane == kWave - 1) wsum[w] = inc;
    __syncthreads();
    int base = 0, tot = 0;
#pragma unroll
    for (int q = 0; q < kWaves; ++q) {
        if (q < w) base += wsum[q];
        tot += wsum[q];
    }
    __syncthreads();
    total = tot;
    return base + inc - v;
}

// Per-block member count (plain store).  With expansion, first folds the
// last round's additions into the round count.
__global__ __launch_bounds__(kBlock) void k_count(const uint8_t *__restrict__ stamp,
                                                  int64_t ntiles, int64_t tiles_per_block,
                                                  int32_t *cnt, int e_max, const double *part_exp,
                                                  int gexp, Scalars *sc) {
    if (e_max >= 1 && !sc->ms.stop) {
        double added[1];
        read_partials<double, 1>(part_exp, gexp, Ops<0u>(), added);
        if (blockIdx.x == 0 && threadIdx.x == 0 && added[0] > 0.0) sc->ms.grown = e_max;
    }
    const int64_t t0 = (int64_t)blockIdx.x * tiles_per_block;
    int64_t t1 = t0 + tiles_per_block;
    if (t1 > ntiles) t1 = ntiles;
    int c = 0;
    const uint64_t *w = reinterpret_cast<const uint64_t *>(stamp);
    for (int64_t t = t0; t < t1; ++t) c += nonzero_bytes(w[t * kBlock + threadIdx.x]);
    __shared__ int red[kWaves];
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) c += __shfl_xor(c, o, kWave);
    if ((threadIdx.x & (kWave - 1)) == 0) red[threadIdx.x / kWave] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        int a = 0;
        for (int q = 0; q < kWaves; ++q) a += red[q];
        cnt[blockIdx.x] = a;
    }
}

// idx[pos] = i for members in ascending i; inv[i] = pos or -1.  Each block
// starts at the sum of the counts of the blocks before it; block 0 records K.
__global__ __launch_bounds__(kBlock) void k_scatter(const uint8_t *__restrict__ stamp, int64_t n,
                                                    int64_t ntiles, int64_t tiles_per_block,
                                                    const int32_t *__restrict__ cnt,
                                                    int32_t *__restrict__ idx,
                                                    int32_t *__restrict__ inv, Scalars *sc) {
    int off, total;
    block_prefix_of_counts(cnt, gridDim.x, blockIdx.x, off, total);
    if (blockIdx.x == 0 && threadIdx.x == 0) sc->ms.K = total;
    const int64_t t0 = (int64_t)blockIdx.x * tiles_per_block;
    int64_t t1 = t0 + tiles_per_block;
    if (t1 > ntiles) t1 = ntiles;
    const uint64_t *w = reinterpret_cast<const uint64_t *>(stamp);
    for (int64_t t = t0; t < t1; ++t) {
        const uint64_t word = w[t * kBlock + threadIdx.x];
        const int c = nonzero_bytes(word);
        int tt;
        int pos = off + block_exclusive_scan(c, tt);
        const int64_t row0 = t * kTile + (int64_t)threadIdx.x * 8;
        if (row0 + 8 <= n) {
            // the thread's 8 rows of inv as two 16-byte stores (row0 is a
            // multiple of 8), so that a wave writes whole lines
            int v[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                if ((word >> (8 * k)) & 0xffull) {
                    idx[pos] = (int32_t)(row0 + k);
                    v[k] = pos++;
                } else {
                    v[k] = -1;
                }
            }
            int4 *o = reinterpret_cast<int4 *>(inv + row0);
            o[0] = make_int4(v[0], v[1], v[2], v[3]);
            o[1] = make_int4(v[4], v[5], v[6], v[7]);
        } else {
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                const int64_t i = row0 + k;
                if (i >= n) break;
                if ((word >> (8 * k)) & 0xffull) {
                    idx[pos] = (int32_t)i;
                    inv[i] = pos;
                    ++pos;
                } else {
                    inv[i] = -1;
                }
            }
        }
        off += tt;
    }
}

// ---------------------------------------------------------------------------
// exclusive scan of int32 (row lengths -> CSR row pointers)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_scan_reduce(const int32_t *__restrict__ in, int64_t n,
                                                        int64_t tiles_per_block, int32_t *blocksum) {
    const int64_t t0 = (int64_t)blockIdx.x * tiles_per_block;
    int s = 0;
    for (int64_t t = t0; t < t0 + tiles_per_block; ++t) {
        const int64_t base = t * kTile + (int64_t)threadIdx.x * 8;
#pragma unroll
        for (int k = 0; k < 8; ++k)
            if (base + k < n) s += in[base + k];
    }
    __shared__ int red[kWaves];
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) s += __shfl_xor(s, o, kWave);
    if ((threadIdx.x & (kWave - 1)) == 0) red[threadIdx.x / kWave] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        int a = 0;
        for (int q = 0; q < kWaves; ++q) a += red[q];
        blocksum[blockIdx.x] = a;
    }
}

// out[i] = sum_{k<i} in[k]; out[n] = total (also recorded as the nnz).
__global__ __launch_bounds__(kBlock) void k_scan_apply(const int32_t *__restrict__ in, int64_t n,
                                                       int64_t tiles_per_block,
                                                       const int32_t *__restrict__ blocksum,
                                                       int32_t *__restrict__ out, Scalars *sc) {
    int off, total;
    block_prefix_of_counts(blocksum, gridDim.x, blockIdx.x, off, total);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        sc->gather_nnz = total;
        out[n] = total;
    }
    const int64_t t0 = (int64_t)blockIdx.x * tiles_per_block;
    for (int64_t t = t0; t < t0 + tiles_per_block; ++t) {
        const int64_t base = t * kTile + (int64_t)threadIdx.x * 8;
        int loc[8];
        int mine = 0;
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            loc[k] = base + k < n ? in[base + k] : 0;
            mine += loc[k];
        }
        int tt;
        int p = off + block_exclusive_scan(mine, tt);
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            if (base + k < n) out[base + k] = p;
            p += loc[k];
        }
        off += tt;
    }
}

// ---------------------------------------------------------------------------
// colour-blocked order of a domain (for the Gauss-Seidel preconditioner)
// ---------------------------------------------------------------------------
// The rows of the restricted system can be put colour by colour, ascending
// inside each colour, so that a colour's half sweep streams only its own
// rows.  Block b takes a contiguous chunk of the ascending domain idx:
// k_cblk_count stores how many of its cells have each colour, and
// k_cblk_place puts cell idx[k] at (cells of lower colours) + (cells of its
// colour in lower blocks) + (its rank among them in its block), writes the
// blocked domain and inv, and the first position of each colour (then K) to
// sc->cstart.
constexpr int kMaxBlkColours = 4;

template <class SOp>
__global__ __launch_bounds__(kBlock) void k_cblk_count(SOp A, const int32_t *__restrict__ idx,
                                                       int64_t K, int64_t chunk, int ncol,
                                                       int32_t *__restrict__ cnt) {
    __shared__ int red[kMaxBlkColours][kWaves];
    const int64_t k0 = (int64_t)blockIdx.x * chunk;
    const int64_t k1 = k0 + chunk < K ? k0 + chunk : K;
    int c[kMaxBlkColours];
#pragma unroll
    for (int q = 0; q < kMaxBlkColours; ++q) c[q] = 0;
    for (int64_t k = k0 + threadIdx.x; k < k1; k += kBlock) {
        const int col = A.colour(idx[k]);
#pragma unroll
        for (int q = 0; q < kMaxBlkColours; ++q) c[q] += col == q ? 1 : 0;
    }
    const int w = threadIdx.x / kWave;
#pragma unroll
    for (int q = 0; q < kMaxBlkColours; ++q) {
        const int t = wave_reduce(c[q], OpSum());
        if ((threadIdx.x & (kWave - 1)) == 0) red[q][w] = t;
    }
    __syncthreads();
    if (threadIdx.x < ncol) {
        int t = 0;
#pragma unroll
        for (int q = 0; q < kWaves; ++q) t += red[threadIdx.x][q];
        cnt[(int64_t)threadIdx.x * gridDim.x + blockIdx.x] = t;
    }
}

// qv (optional, two colours): at each row's position, the position the
// other colour's block gives a cell at the row's grid index (UEllRB's q).
template <class SOp>
__global__ __launch_bounds__(kBlock) void k_cblk_place(SOp A, const int32_t *__restrict__ idx,
                                                       int64_t K, int64_t chunk, int ncol,
                                                       const int32_t *__restrict__ cnt,
                                                       int32_t *__restrict__ idxb,
                                                       int32_t *__restrict__ inv, Scalars *sc,
                                                       int32_t *__restrict__ qv) {
    int64_t base[kMaxBlkColours];
    int64_t lower = 0;   // cells of the colours below q
#pragma unroll
    for (int q = 0; q < kMaxBlkColours; ++q) {
        base[q] = 0;
        if (q < ncol) {
            int before = 0, total = 0;
            block_prefix_of_counts(cnt + (int64_t)q * gridDim.x, gridDim.x, blockIdx.x, before,
                                   total);
            base[q] = lower + before;
            if (blockIdx.x == 0 && threadIdx.x == 0) sc->cstart[q] = lower;
            lower += total;
        }
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) sc->cstart[ncol] = lower;
    const int64_t k0 = (int64_t)blockIdx.x * chunk;
    const int64_t k1 = k0 + chunk < K ? k0 + chunk : K;
    for (int64_t t0 = k0; t0 < k1; t0 += kBlock) {
        const int64_t k = t0 + threadIdx.x;
        const int32_t i = k < k1 ? idx[k] : 0;
        const int col = k < k1 ? A.colour(i) : -1;
        int64_t own = 0, other = 0;
#pragma unroll
        for (int q = 0; q < kMaxBlkColours; ++q) {
            if (q < ncol) {
                int tot = 0;
                const int pre = block_exclusive_scan(col == q ? 1 : 0, tot);
                if (col == q) {
                    const int64_t pos = base[q] + pre;
                    idxb[pos] = i;
                    inv[i] = (int32_t)pos;
                    own = pos;
                } else {
                    other = base[q] + pre;
                }
                base[q] += tot;
            }
        }
        if (qv && col >= 0) qv[own] = (int32_t)other;
    }
}

// ---------------------------------------------------------------------------
// restricted system B = A[Omega, Omega] (eq. BEFC)
// ---------------------------------------------------------------------------
// Row k of B (global row idx[k]) in column-major ELL of width W: members in
// ascending column order (columns renumbered through inv, which keeps the
// order), then col = -1.  Also the diagonal, the colour of the row and
// rhs_B = r^(0)_Omega (right-hand side of the correction form of eq. loc-equ).
template <class Op>
__global__ __launch_bounds__(kBlock) void k_gather_ell(
    Op A, const int32_t *__restrict__ idx, int64_t K, const int32_t *__restrict__ inv, int W,
    int32_t *__restrict__ col, double *__restrict__ val, float *__restrict__ val32,
    double *__restrict__ dg, float *__restrict__ dg32, uint8_t *__restrict__ clr,
    const double *__restrict__ r, double *__restrict__ rhs) {
    for (int64_t k = blockIdx.x * (int64_t)kBlock + threadIdx.x; k < K;
         k += (int64_t)gridDim.x * kBlock) {
        const int64_t i = idx[k];
        int t = 0;
        A.for_each(i, [&](int64_t j, double a) {
            const int32_t cj = inv[j];
            if (cj >= 0) {
                col[t * K + k] = cj;
                val[t * K + k] = a;
                if (val32) val32[t * K + k] = (float)a;
                ++t;
            }
        });
        for (; t < W; ++t) {
            col[t * K + k] = -1;
            val[t * K + k] = 0.0;
            if (val32) val32[t * K + k] = 0.0f;
        }
        const double d = A.diag(i);
        dg[k] = d;
        if (dg32) dg32[k] = (float)d;
        clr[k] = (uint8_t)A.colour(i);
        if (rhs) rhs[k] = r[i];
    }
}

// The same B in UEllShort's form (a domain in grid order on the five- or
// nine-point stencil): the values of the upper slots (C and above, zero
// where the neighbour is not a member), each row's presence bits and the offsets
// soff / noff of the number of members before the cell straight below /
// above (found from whichever of the cells below / above are members; zero
// when none is).
template <class Op>
__global__ __launch_bounds__(kBlock) void k_gather_rowcode(
    Op A, const int32_t *__restrict__ idx, int64_t K, const int32_t *__restrict__ inv,
    uint32_t *__restrict__ off, uint8_t *__restrict__ mask,
    double *__restrict__ val, float *__restrict__ val32, double *__restrict__ dg,
    float *__restrict__ dg32, uint8_t *__restrict__ clr, const double *__restrict__ r,
    double *__restrict__ rhs) {
    constexpr int NB = Op::kSlots, kMid = NB / 2;
    for (int64_t k = blockIdx.x * (int64_t)kBlock + threadIdx.x; k < K;
         k += (int64_t)gridDim.x * kBlock) {
        const int64_t i = idx[k];
        int32_t cs[NB];
        double a[NB];
#pragma unroll
        for (int sl = 0; sl < NB; ++sl) {
            cs[sl] = -1;
            a[sl] = 0.0;
        }
        A.for_each_slot(i, [&](int sl, int64_t j, double v) {
            const int32_t cj = inv[j];
            if (cj >= 0) {
                cs[sl] = cj;
                a[sl] = v;
            }
        });
        unsigned m = 0;
#pragma unroll
        for (int sl = 0; sl < NB; ++sl) {
            if (sl != kMid && cs[sl] >= 0) m |= 1u << (sl < kMid ? sl : sl - 1);
            if (sl >= kMid) {
                val[(sl - kMid) * K + k] = a[sl];
                if (val32) val32[(sl - kMid) * K + k] = (float)a[sl];
            }
        }
        int64_t ps = k, pn = k;
        if constexpr (NB == 9) {
            ps = cs[0] >= 0 ? cs[0] + 1 : cs[1] >= 0 ? cs[1] : cs[2] >= 0 ? cs[2] : k;
            pn = cs[6] >= 0 ? cs[6] + 1 : cs[7] >= 0 ? cs[7] : cs[8] >= 0 ? cs[8] : k;
        } else {
            ps = cs[0] >= 0 ? cs[0] : k;
            pn = cs[4] >= 0 ? cs[4] : k;
        }
        off[k] = (uint32_t)(uint16_t)(int16_t)(ps - k) | (uint32_t)(uint16_t)(int16_t)(pn - k) << 16;
        mask[k] = (uint8_t)m;
        const double d = A.diag(i);
        dg[k] = d;
        if (dg32) dg32[k] = (float)d;
        clr[k] = (uint8_t)A.colour(i);
        if (rhs) rhs[k] = r[i];
    }
}

// The red-black colour-blocked B in UEllRB's form: rows in the blocked
// order idx (k_cblk_place's, which left each row's q in code.q), values in
// the stencil's fixed slots, presence bits and the distances from q to the
// members below and above.
template <class Op>
__global__ __launch_bounds__(kBlock) void k_gather_rbcode(
    Op A, const int32_t *__restrict__ idx, int64_t K, const int32_t *__restrict__ inv,
    const int32_t *__restrict__ qv, uint64_t *__restrict__ dw, uint8_t *__restrict__ mask,
    double *__restrict__ val, float *__restrict__ val32, double *__restrict__ dg,
    float *__restrict__ dg32, uint8_t *__restrict__ clr, const double *__restrict__ r,
    double *__restrict__ rhs) {
    constexpr int NB = Op::kSlots, kMid = NB / 2;
    for (int64_t k = blockIdx.x * (int64_t)kBlock + threadIdx.x; k < K;
         k += (int64_t)gridDim.x * kBlock) {
        const int64_t i = idx[k];
        const int64_t q = qv[k];
        int32_t cs[NB];
        double a[NB];
#pragma unroll
        for (int sl = 0; sl < NB; ++sl) {
            cs[sl] = -1;
            a[sl] = 0.0;
        }
        A.for_each_slot(i, [&](int sl, int64_t j, double v) {
            const int32_t cj = inv[j];
            if (cj >= 0) {
                cs[sl] = cj;
                a[sl] = v;
            }
        });
        unsigned m = 0;
#pragma unroll
        for (int sl = 0; sl < NB; ++sl) {
            if (sl != kMid && cs[sl] >= 0) m |= 1u << (sl < kMid ? sl : sl - 1);
            val[sl * K + k] = a[sl];
            if (val32) val32[sl * K + k] = (float)a[sl];
        }
        uint64_t ds = 0, dn = 0, dd = 0, du = 0;
        if constexpr (NB == 7) {
            dd = (uint64_t)(cs[0] >= 0 ? q - cs[0] : 0);
            ds = (uint64_t)(cs[1] >= 0 ? q - cs[1] : 0);
            dn = (uint64_t)(cs[5] >= 0 ? cs[5] - q : 0);
            du = (uint64_t)(cs[6] >= 0 ? cs[6] - q : 0);
        } else {
            ds = (uint64_t)(cs[0] >= 0 ? q - cs[0] : 0);
            dn = (uint64_t)(cs[4] >= 0 ? cs[4] - q : 0);
        }
        dw[k] = ds | dn << 16 | dd << 32 | du << 48;
        mask[k] = (uint8_t)m;
        const double d = A.diag(i);
        dg[k] = d;
        if (dg32) dg32[k] = (float)d;
        clr[k] = (uint8_t)A.colour(i);
        if (rhs) rhs[k] = r[i];
    }
}

// row lengths of the ELL form (members = col >= 0)
__global__ __launch_bounds__(kBlock) void k_ell_rowlen(const int32_t *__restrict__ col, int64_t K,
                                                       int W, int32_t *__restrict__ len) {
    for (int64_t k = blockIdx.x * (int64_t)kBlock + threadIdx.x; k < K;
         k += (int64_t)gridDim.x * kBlock) {
        int c = 0;
        for (int t = 0; t < W; ++t) c += col[t * K + k] >= 0;
        len[k] = c;
    }
}

// ELL -> CSR (row pointers from the scan)
__global__ __launch_bounds__(kBlock) void k_ell_to_csr(const int32_t *__restrict__ ecol,
                                                       const double *__restrict__ eval, int64_t K,
                                                       int W, const int32_t *__restrict__ rp,
                                                       int32_t *__restrict__ col,
                                                       double *__restrict__ val) {
    for (int64_t k = blockIdx.x * (int64_t)kBlock + threadIdx.x; k < K;
         k += (int64_t)gridDim.x * kBlock) {
        int32_t o = rp[k];
        for (int t = 0; t < W; ++t) {
            const int32_t c = ecol[t * K + k];
            if (c < 0) break;
            col[o] = c;
            val[o] = eval[t * K + k];
            ++o;
        }
    }
}

// inv[idx[k]] = k for a caller-supplied domain (inv pre-filled with -1).
// Entries out of [0, n) or not strictly ascending are skipped and flagged.
__global__ __launch_bounds__(kBlock) void k_set_inv(const int32_t *__restrict__ idx, int64_t K,
                                                    int64_t n, int32_t *__restrict__ inv,
                                                    Scalars *sc) {
    for (int64_t k = blockIdx.x * (int64_t)kBlock + threadIdx.x; k < K;
         k += (int64_t)gridDim.x * kBlock) {
        const int32_t i = idx[k];
        const bool ok = i >= 0 && i < n && (k == 0 || idx[k - 1] < i);
        if (ok) inv[i] = (int32_t)k;
        else atomicOr(&sc->bad_idx, 1);
    }
}

// x[idx[k]] += d[k]  (eq. sol-assemble in correction form); x2 (optional,
// a copy of x) gets the same new values.
__global__ __launch_bounds__(kBlock) void k_scatter_add(const int32_t *__restrict__ idx,
                                                        const double *__restrict__ d, int64_t K,
                                                        double *__restrict__ x,
                                                        double *__restrict__ x2) {
    for (int64_t k = blockIdx.x * (int64_t)kBlock + threadIdx.x; k < K;
         k += (int64_t)gridDim.x * kBlock) {
        const int64_t i = idx[k];
        const double v = x[i] + d[k];
        x[i] = v;
        if (x2) x2[i] = v;
    }
}

// ---------------------------------------------------------------------------
// preconditioned CG (templated on operator and working precision)
// ---------------------------------------------------------------------------
// Iteration j is the pair k_pcg_ap(j), k_pcg_update(j) (plus the
// Gauss-Seidel half sweeps for RB-SGS).  Each kernel starts by folding the
// partials of the kernel before it, so every block holds the same scalars;
// block 0 records them for later kernels and the host.
//
// RB-SGS applies the symmetric colour-ordered sweeps 0, 1, .., c-1, .., 1, 0
// to M z = r from z = 0.  The first sweep, over colour 0 with every
// neighbour still zero, is z_i = r_i / a_ii exactly (each fma(-a, 0, acc)
// leaves acc unchanged), so the kernels that form r also do it; the host
// launches the remaining sweeps from colour 1.
//
// init: r = rhs - A x (or r = rhs when x = 0); Jacobi: z = r / a_ii; none:
// z = r; RB-SGS: z = r / a_ii on colour 0, else 0.  Partials r.r, r.z.
template <class Op, int kPc>
__global__ __launch_bounds__(kBlock) void k_pcg_init(Op A, const typename Op::real *__restrict__ rhs,
                                                     const typename Op::real *__restrict__ x,
                                                     typename Op::real *__restrict__ r,
                                                     typename Op::real *__restrict__ z, int x_zero,
                                                     Scalars *sc, typename Op::real *part_upd) {
    using real = typename Op::real;
    constexpr int V = Op::V, NB = Op::NB;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        sc->pcg.done = 0;
        sc->pcg.status = kStOk;
        sc->pcg.it = 0;
    }
    real v[2] = {real(0), real(0)};
    for (auto W = walk<1>(A); W.valid(); W.advance()) {
        typename Op::Unit U;
        real rr[V], zz[V];
        if (x_zero) {
            W.geom(A, U);
            A.own(U, rhs, rr);
        } else {
            W.load(A, U);
            real xv[NB][V], bb[V];
            W.template gather<0>(A, U, x, xv);
            A.own(U, rhs, bb);
#pragma unroll
            for (int k = 0; k < V; ++k) {
                real acc = bb[k];
#pragma unroll
                for (int q = 0; q < NB; ++q)
                    if (A.valid(U, q, k)) acc = fma(-U.a[q][k], xv[q][k], acc);
                rr[k] = acc;
            }
        }
        if (kPc >= 1) {
            real d[V];
            A.diag(U, d);
#pragma unroll
            for (int k = 0; k < V; ++k)
                zz[k] = (kPc == 1 || A.colour(U, k) == 0) ? rr[k] / d[k] : real(0);
        } else {
#pragma unroll
            for (int k = 0; k < V; ++k) zz[k] = rr[k];
        }
        A.put(U, r, rr);
        A.put(U, z, zz);
#pragma unroll
        for (int k = 0; k < V; ++k) {
            v[0] += rr[k] * rr[k];
            v[1] += rr[k] * zz[k];
        }
    }
    write_partials<real, 2>(v, Ops<0u>(), part_upd);
}

// Iteration j, first kernel.  Prologue: r_j.r_j and r_j.z_j from the
// previous kernel's partials -> stop (criterion, max_iter, non-finite), else
// beta_j = r_j.z_j / r_{j-1}.z_{j-1}.  Body: q = A p with p = z (j = 0) or
// p = z + beta p_old, recomputed for each neighbour so that p is updated in
// the same pass (p_new written for the own cells only).  Partials p.q.
template <class Op, int kPc>
__global__ __launch_bounds__(kBlock) void k_pcg_ap(Op A, const typename Op::real *__restrict__ z,
                                                   const typename Op::real *__restrict__ pold,
                                                   typename Op::real *__restrict__ pnew,
                                                   typename Op::real *__restrict__ q, int j,
                                                   int max_iter, const double *tol_base,
                                                   double tol_factor, Scalars *sc,
                                                   const typename Op::real *part_upd,
                                                   const typename Op::real *part_sgs, int gsgs,
                                                   typename Op::real *part_ap) {
    using real = typename Op::real;
    constexpr int V = Op::V, NB = Op::NB;
    // scalars, stop flag and the first unit's coefficients before the fold
    // (their latencies overlap; see k_cg_iter)
    const int done = sc->pcg.done;
    const double tol_prev = sc->pcg.tol, rz_prev = sc->pcg.rz_cur;
    const double tol_in = (j == 0 && tol_base) ? *tol_base : 0.0;
    auto W = walk<2>(A);
    typename Op::Unit U;
    if (W.valid()) W.load(A, U);
    real t[2];
    read_partials<real, 2>(part_upd, gridDim.x, Ops<0u>(), t);
    real rz = t[1];
    if (kPc == 2) {
        real u[1];
        read_partials<real, 1>(part_sgs, gsgs, Ops<0u>(), u);
        rz = u[0];
    }
    if (done) return;
    const double rr = (double)t[0];
    double tol;
    if (j == 0) tol = tol_base ? tol_factor * tol_in : tol_factor * sqrt(rr);
    else tol = tol_prev;
    int stop = 0, status = kStOk;
    if (!(rr == rr) || rr > 1.7e308) {
        stop = 1;
        status = kStNonFinite;
    } else if (sqrt(rr) <= tol) {
        stop = 1;
    } else if (j >= max_iter) {
        stop = 1;
        status = kStNoConv;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        if (j == 0) {
            sc->pcg.tol = tol;
            sc->pcg.rr0 = rr;
        }
        sc->pcg.rr = rr;
        sc->pcg.rz_next = (double)rz;
        if (stop) {
            sc->pcg.done = 1;
            sc->pcg.status = status;
            sc->pcg.it = j;
        }
    }
    if (stop) return;
    const real beta = j == 0 ? real(0) : rz / (real)rz_prev;
    real v[1] = {real(0)};
    for (bool first = true; W.valid(); W.advance(), first = false) {
        if (!first) W.load(A, U);
        real pv[NB][V], po[V], zo[V];
        W.template gather<0>(A, U, z, pv);
        own_of(A, U, pv, z, zo);
        if (j == 0) {
#pragma unroll
            for (int k = 0; k < V; ++k) po[k] = zo[k];
        } else {
            real ov[NB][V], oo[V];
            W.template gather<1>(A, U, pold, ov);
            own_of(A, U, ov, pold, oo);
#pragma unroll
            for (int q = 0; q < NB; ++q)
#pragma unroll
                for (int k = 0; k < V; ++k) pv[q][k] = fma(beta, ov[q][k], pv[q][k]);
#pragma unroll
            for (int k = 0; k < V; ++k) po[k] = fma(beta, oo[k], zo[k]);
        }
        real qq[V];
#pragma unroll
        for (int k = 0; k < V; ++k) {
            real acc = real(0);
#pragma unroll
            for (int s2 = 0; s2 < NB; ++s2)
                if (A.valid(U, s2, k)) acc = fma(U.a[s2][k], pv[s2][k], acc);
            qq[k] = acc;
            v[0] += po[k] * acc;
        }
        A.put(U, pnew, po);
        A.put(U, q, qq);
    }
    write_partials<real, 1>(v, Ops<0u>(), part_ap);
}

// Iteration j, second kernel.  Prologue: p.q from the partials ->
// breakdown if p.q <= 0, else alpha = r.z / p.q.  Body: x += alpha p;
// r -= alpha q; Jacobi z = r / a_ii (none: z = r; RB-SGS: the colour-0 sweep
// from z = 0, as in init).  Partials r.r, r.z.
template <class Op, int kPc>
__global__ __launch_bounds__(kBlock) void k_pcg_update(Op A, typename Op::real *__restrict__ x,
                                                       const typename Op::real *__restrict__ p,
                                                       const typename Op::real *__restrict__ q,
                                                       typename Op::real *__restrict__ r,
                                                       typename Op::real *__restrict__ z, int j,
                                                       Scalars *sc, const typename Op::real *part_ap,
                                                       typename Op::real *part_upd) {
    using real = typename Op::real;
    constexpr int V = Op::V;
    // stop flag, r.z and the first unit's vectors before the partial fold
    // (their latencies overlap; see k_cg_iter)
    const int done = sc->pcg.done;
    const double rzd = sc->pcg.rz_next;
    Band B = my_band(A.units());
    typename Op::Unit U;
    real xx[V], pp[V], qq[V], rr[V], zz[V], d[V];
    auto load_unit = [&](int64_t u) {
        A.geom(U, u);
        A.own(U, x, xx);
        A.own(U, p, pp);
        A.own(U, q, qq);
        A.own(U, r, rr);
        if (kPc >= 1) A.diag(U, d);
    };
    if (B.u < B.end) load_unit(B.u);
    real t[1];
    read_partials<real, 1>(part_ap, gridDim.x, Ops<0u>(), t);
    if (done) return;
    const double pq = (double)t[0];
    if (!(pq > 0.0)) {
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            sc->pcg.done = 1;
            sc->pcg.status = (pq == pq) ? kStBreakdown : kStNonFinite;
            sc->pcg.it = j;
        }
        return;
    }
    const real alpha = (real)rzd / t[0];
    if (blockIdx.x == 0 && threadIdx.x == 0) sc->pcg.rz_cur = rzd;
    real v[2] = {real(0), real(0)};
    for (bool first = true; B.u < B.end; B.u += B.step, first = false) {
        if (!first) load_unit(B.u);
#pragma unroll
        for (int k = 0; k < V; ++k) {
            xx[k] = fma(alpha, pp[k], xx[k]);
            rr[k] = fma(-alpha, qq[k], rr[k]);
            zz[k] = kPc == 0 ? rr[k] : (kPc == 1 || A.colour(U, k) == 0) ? rr[k] / d[k] : real(0);
            v[0] += rr[k] * rr[k];
            v[1] += rr[k] * zz[k];
        }
        A.put(U, x, xx);
        A.put(U, r, rr);
        A.put(U, z, zz);
    }
    write_partials<real, 2>(v, Ops<0u>(), part_upd);
}

// One Gauss-Seidel half sweep over colour c: for cells of that colour,
// z_i = (r_i - sum_{j != i, ascending} a_ij z_j) / a_ii.  Cells of one
// colour never couple, so the update is order-free.  With kRz the kernel
// also writes partials of r.z (all cells).  With a null state this is the
// smoother of Algorithm 1 (r = b, z = x).
template <class Op, bool kRz>
__global__ __launch_bounds__(kBlock) void k_gs_half(Op A, const typename Op::real *__restrict__ r,
                                                    typename Op::real *z, int colour,
                                                    const Scalars *sc, typename Op::real *part_sgs) {
    using real = typename Op::real;
    constexpr int V = Op::V, NB = Op::NB;
    if (sc && sc->pcg.done) return;
    real v[1] = {real(0)};
    for (auto W = walk<1>(A); W.valid(); W.advance()) {
        typename Op::Unit U;
        W.load(A, U);
        real zv[NB][V], ro[V], zo[V];
        W.template gather<0>(A, U, (const real *)z, zv);
        A.own(U, r, ro);
        own_of(A, U, zv, (const real *)z, zo);
        bool any = false;
#pragma unroll
        for (int k = 0; k < V; ++k) {
            if (A.colour(U, k) == colour) {
                real acc = ro[k], d = real(1);
#pragma unroll
                for (int q = 0; q < NB; ++q) {
                    if (!A.valid(U, q, k)) continue;
                    if (A.is_diag(U, q, k)) d = U.a[q][k];
                    else acc = fma(-U.a[q][k], zv[q][k], acc);
                }
                zo[k] = acc / d;
                any = true;
            }
            if (kRz) v[0] += ro[k] * zo[k];
        }
        if (any) A.put(U, z, zo);
    }
    if (kRz) write_partials<real, 1>(v, Ops<0u>(), part_sgs);
}

// The half sweep of colour c on a restricted system whose rows are blocked
// by colour (rows [a, b) have colour c): only those rows are read and
// updated, each with k_gs_half's arithmetic, so the z it leaves is the same
// bit for bit.  With kRz this is the colour's last update of the sweep
// pair, and the kernel writes the partials of r.z over its rows (one
// partial set per colour; the consumer folds all of them).
template <class Op, bool kRz>
__global__ __launch_bounds__(kBlock) void k_gs_half_blk(Op A, const typename Op::real *__restrict__ r,
                                                        typename Op::real *z, int64_t a, int64_t b,
                                                        const Scalars *sc, typename Op::real *part_sgs) {
    using real = typename Op::real;
    constexpr int NB = Op::NB;
    static_assert(Op::V == 1, "rows of the restricted system");
    if (sc->pcg.done) return;
    real v[1] = {real(0)};
    const Band B = my_band(b - a);
    for (int64_t u = B.u; u < B.end; u += B.step) {
        const int64_t i = u + a;
        typename Op::Unit U;
        A.load(U, i);
        real zv[NB][1], ro[1], zo[1];
        A.gather(U, (const real *)z, zv);
        A.own(U, r, ro);
        real acc = ro[0], d = real(1);
#pragma unroll
        for (int q = 0; q < NB; ++q) {
            if (!A.valid(U, q, 0)) continue;
            if (A.is_diag(U, q, 0)) d = U.a[q][0];
            else acc = fma(-U.a[q][0], zv[q][0], acc);
        }
        zo[0] = acc / d;
        A.put(U, z, zo);
        if (kRz) v[0] += ro[0] * zo[0];
    }
    if (kRz) write_partials<real, 1>(v, Ops<0u>(), part_sgs);
}

// Two colours of the four-colour Gauss-Seidel sweep of the nine-point
// stencil (colour (x mod 2) + 2 (y mod 2)) in one pass.  The rows of parity p
// hold colours 2p (x even) and 2p+1 (x odd), and nothing else: rows of one
// parity never couple to each other, colour 2p reads only the other parity's
// rows and colour 2p+1 of its own row, and colour 2p+1 reads the new colour
// 2p of its own row (x - 1, x + 1) and the other parity's rows.  So the
// sweep over colours 0, 1, 2, 3 is the pass p = 0 then the pass p = 1, with
// per-cell results identical to four one-colour kernels: the same FMA chain
// in ascending slot order over the same old and new values.
//
// The pass reads x from `in` and writes every row to `out`: rows of parity
// p with their new values, the other rows copied.  Reading one buffer and
// writing another keeps the old values of a row that a neighbouring wave
// may be updating.  A wave owns 63 strips of V = 2 cells of a row (lanes
// 0..62) and walks up mh rows; lane 63 holds the next strip's first unit,
// whose new colour-2p value its left neighbour needs, and stores nothing.
// Per own row a lane loads its row's five coefficient arrays, the three
// south arrays of the row below, and the rows y and y+1 of x (row y-1 is
// carried); every array element is read about once per pass.
constexpr int kPairStep = kWave - 1;

template <class Op>
__global__ __launch_bounds__(kBlock) void k_gs_pair9(Op A, const double *__restrict__ b,
                                                     const double *__restrict__ in,
                                                     double *__restrict__ out, int parity, int mh) {
    static_assert(Op::V == 2 && Op::NB == 9, "nine-point strips of two cells");
    constexpr int V = 2;
    using Unit = typename Op::Unit;
    const int lane = threadIdx.x % kWave;
    const int nx = A.nx, ny = A.ny;
    const int64_t upr = nx / V;
    const int64_t strips = (upr + kPairStep - 1) / kPairStep;
    const int64_t tiles = strips * (int64_t)((ny + mh - 1) / mh);
    for (int64_t t = (int64_t)logical_block() * kWaves + threadIdx.x / kWave; t < tiles;
         t += (int64_t)gridDim.x * kWaves) {
        const int64_t strip = t % strips, seg = t / strips;
        const int64_t xr = strip * kPairStep + lane;
        const bool active = xr < upr;
        const bool owner = active && lane < kPairStep;
        const int xu = (int)(active ? xr : upr - 1);   // lanes past the row end load a valid strip
        const int x0 = xu * V;
        const int y0 = (int)seg * mh, y1 = min(ny, y0 + mh);
        double xs[V + 2], xc[V + 2], xn[V + 2];
        int y = y0;
        bool carried = false;
        if ((y0 & 1) != parity) {   // a leading row of the other parity: copied
            const int64_t i = (int64_t)y0 * nx + x0;
            row_load<double, V>(in, i, i, x0, nx, true, true, xs);
            if (owner) vst<double, V>(out + i, {xs[1], xs[2]});
            carried = true;
            ++y;
        }
        for (; y < y1; y += 2) {
            const int64_t i0 = (int64_t)y * nx + x0;
            if (!carried) row_load<double, V>(in, i0 - nx, i0, x0, nx, y > 0, true, xs);
            row_load<double, V>(in, i0, i0, x0, nx, true, true, xc);
            row_load<double, V>(in, i0 + nx, i0, x0, nx, y + 1 < ny, true, xn);
            if (owner && y + 1 < y1) vst<double, V>(out + i0 + nx, {xn[1], xn[2]});
            Unit U;
            A.geom_walk(U, (int64_t)y * upr + xu, xu, y);
            typename Op::South S;
            A.south_init(S, U);
            A.load_row(U, S);
            double bb[V];
            vld<double, V>(b + i0, bb);
            double nv[V];
#pragma unroll
            for (int k = 0; k < V; ++k) {
                double z[9];
                z[0] = xs[k]; z[1] = xs[k + 1]; z[2] = xs[k + 2];
                z[3] = xc[k]; z[4] = xc[k + 1]; z[5] = xc[k + 2];
                z[6] = xn[k]; z[7] = xn[k + 1]; z[8] = xn[k + 2];
                if (k == 1) {
                    z[3] = nv[0];                           // colour 2p at x0, new
                    z[5] = __shfl_down(nv[0], 1, kWave);    // colour 2p at x0 + 2, new
                }
                double acc = bb[k], d = 1.0;
#pragma unroll
                for (int q = 0; q < 9; ++q) {
                    if (!A.valid(U, q, k)) continue;
                    if (q == Op::kC) d = U.a[q][k];
                    else acc = fma(-U.a[q][k], z[q], acc);
                }
                nv[k] = acc / d;
            }
            if (owner) vst<double, V>(out + i0, nv);
#pragma unroll
            for (int k = 0; k < V + 2; ++k) xs[k] = xn[k];
            carried = true;
        }
    }
}

// The pass p of k_gs_pair9 fused with the criterion after it (Algorithm 1
// step 8): besides the pass's output it forms r = b - A x over the whole grid
// from the values the pass leaves, per cell with k_resnorm's FMA chain, and
// writes k_resnorm's partials (||r||^2, max|r|) for k_fin_res.  Rows are
// visited one at a time, up from y0 - 1 to y1: the tile's rows of parity p
// are updated and stored, the others copied; a row's residual takes its
// slots 0..5 once the row itself is final and slots 6..8 one step later,
// which keeps k_resnorm's order and carries two values instead of the
// row's coefficients.  The rows y0 - 1
// and y1 belong to the neighbouring tiles; when they have parity p the tile
// updates them too, without storing, so that its residuals read final
// values only.  In a row, lanes 1..62 own strips; lanes 0 and 63 update the
// strips on either side (the new value at x0 - 1 of lane 1 and at x0 + 2 of
// lane 62) and store nothing.  Each row reads x, the five coefficient arrays
// and b once (the south faces are carried), and writes x once.
constexpr int kPairOwn = kWave - 2;

template <class Op>
__global__ __launch_bounds__(kBlock) void k_gs_pair9_res(Op A, const double *__restrict__ b,
                                                         const double *__restrict__ in,
                                                         double *__restrict__ out, int parity,
                                                         int mh, double *part) {
    static_assert(Op::V == 2 && Op::NB == 9, "nine-point strips of two cells");
    constexpr int V = 2;
    using Unit = typename Op::Unit;
    const int lane = threadIdx.x % kWave;
    const int nx = A.nx, ny = A.ny;
    const int64_t upr = nx / V;
    const int64_t strips = (upr + kPairOwn - 1) / kPairOwn;
    const int64_t tiles = strips * (int64_t)((ny + mh - 1) / mh);
    double v[2] = {0.0, 0.0};
    for (int64_t t = (int64_t)logical_block() * kWaves + threadIdx.x / kWave; t < tiles;
         t += (int64_t)gridDim.x * kWaves) {
        const int64_t strip = t % strips, seg = t / strips;
        const int64_t xr = strip * kPairOwn + lane - 1;
        const bool active = xr >= 0 && xr < upr;
        const bool owner = active && lane >= 1 && lane <= kPairOwn;
        // lanes outside the row load a valid strip; what they compute is
        // read only for neighbours outside the grid, whose slots are invalid
        const int xu = (int)(xr < 0 ? 0 : (xr >= upr ? upr - 1 : xr));
        const int x0 = xu * V;
        const int y0 = (int)seg * mh, y1 = min(ny, y0 + mh);
        // carried: old rows y-1 and y of `in`; the final row y-1; the
        // south faces of row y (the N, NE, NW arrays of row y-1); and row
        // y-1's residual over its slots 0..5, finished with slots 6..8 once
        // row y holds its final values
        double om[V + 2], oc[V + 2], fm1[V + 2], accp[V];
        {
            const int ya = y0 - 2, yb = y0 - 1;
            const int64_t sa = (int64_t)max(ya, 0) * nx + x0, sb = (int64_t)max(yb, 0) * nx + x0;
            row_load<double, V>(in, sa, sa, x0, nx, ya >= 0, true, om);
            row_load<double, V>(in, sb, sb, x0, nx, yb >= 0, true, oc);
        }
#pragma unroll
        for (int k = 0; k < V + 2; ++k) fm1[k] = 0.0;
#pragma unroll
        for (int k = 0; k < V; ++k) accp[k] = 0.0;
        typename Op::South S;
#pragma unroll
        for (int k = 0; k < V; ++k) S.n[k] = 0.0;
#pragma unroll
        for (int k = 0; k <= V; ++k) S.ne[k] = S.nw[k] = 0.0;
        for (int y = y0 - 1; y <= y1; ++y) {
            const bool real = y >= 0 && y < ny;
            const int yn = y + 1;
            const int64_t sn = (int64_t)min(max(yn, 0), ny - 1) * nx + x0;
            double on[V + 2];
            row_load<double, V>(in, sn, sn, x0, nx, yn >= 0 && yn < ny, true, on);
            // slots 6..8 (NW, N, NE) of row y-1 are the south faces of row
            // y, which row y's load puts into its slots 0..2; the two that
            // fall outside those (NW at x0, NE at x0 + 2) are kept first
            static_assert(V == 2, "the face bookkeeping below is for strips of two");
            const double nw_x0 = S.nw[0], ne_x2 = S.ne[2];
            Unit U;
            U.x0 = x0;
            U.y = y;
            double bb[V] = {0.0, 0.0};
            if (real) {
                A.geom_walk(U, (int64_t)y * upr + xu, xu, y);
                if (y == max(y0 - 1, 0)) A.south_init(S, U);
                A.load_row(U, S);
                vld<double, V>(b + U.i0, bb);
            }
            double f0[V + 2];
            if (real && (y & 1) == parity) {
                // colour 2p, then 2p+1 with the new 2p values of its row
                double nv[V];
#pragma unroll
                for (int k = 0; k < V; ++k) {
                    double z[9];
                    z[0] = om[k]; z[1] = om[k + 1]; z[2] = om[k + 2];
                    z[3] = oc[k]; z[4] = oc[k + 1]; z[5] = oc[k + 2];
                    z[6] = on[k]; z[7] = on[k + 1]; z[8] = on[k + 2];
                    if (k == 1) {
                        z[3] = nv[0];
                        z[5] = __shfl_down(nv[0], 1, kWave);
                    }
                    double acc = bb[k], d = 1.0;
#pragma unroll
                    for (int q = 0; q < 9; ++q) {
                        if (!A.valid(U, q, k)) continue;
                        if (q == Op::kC) d = U.a[q][k];
                        else acc = fma(-U.a[q][k], z[q], acc);
                    }
                    nv[k] = acc / d;
                }
                f0[0] = __shfl_up(nv[1], 1, kWave);
                f0[1] = nv[0];
                f0[2] = nv[1];
                f0[3] = __shfl_down(nv[0], 1, kWave);
            } else {
#pragma unroll
                for (int k = 0; k < V + 2; ++k) f0[k] = oc[k];
            }
            if (owner && y >= y0 && y < y1) vst<double, V>(out + U.i0, {f0[1], f0[2]});
            if (owner && y - 1 >= y0 && y - 1 < y1) {
                // row y-1's residual: its slots 6..8 over the final row y
                Unit Ug;
                Ug.x0 = x0;
                Ug.y = y - 1;
                // row y-1's NW, N, NE at x0 + k: k = 0: (nw_x0, a[1][0],
                // a[0][1]); k = 1: (a[2][0], a[1][1], ne_x2)
                const double a6[V] = {nw_x0, U.a[2][0]};
                const double a7[V] = {U.a[1][0], U.a[1][1]};
                const double a8[V] = {U.a[0][1], ne_x2};
#pragma unroll
                for (int k = 0; k < V; ++k) {
                    double acc = accp[k];
                    if (A.valid(Ug, 6, k)) acc = fma(-a6[k], f0[k], acc);
                    if (A.valid(Ug, 7, k)) acc = fma(-a7[k], f0[k + 1], acc);
                    if (A.valid(Ug, 8, k)) acc = fma(-a8[k], f0[k + 2], acc);
                    v[0] += acc * acc;
                    const double m = fabs(acc);
                    v[1] = m > v[1] ? m : v[1];
                }
            }
            // row y's residual over its slots 0..5 (the final rows y-1, y),
            // in k_resnorm's order
#pragma unroll
            for (int k = 0; k < V; ++k) {
                double z[6];
                z[0] = fm1[k]; z[1] = fm1[k + 1]; z[2] = fm1[k + 2];
                z[3] = f0[k];  z[4] = f0[k + 1];  z[5] = f0[k + 2];
                double acc = bb[k];
#pragma unroll
                for (int q = 0; q < 6; ++q)
                    if (real && A.valid(U, q, k)) acc = fma(-U.a[q][k], z[q], acc);
                accp[k] = acc;
            }
#pragma unroll
            for (int k = 0; k < V + 2; ++k) {
                fm1[k] = f0[k];
                om[k] = oc[k];
                oc[k] = on[k];
            }
        }
    }
    write_partials<double, 2>(v, Ops<2u>(), part);
}

// A whole four-colour sweep of the nine-point stencil in one pass, with the
// criterion's residual after it when kRes (Algorithm 1 steps 7 and 8).  A
// tile visits its even rows going up; at even row y it updates row y
// (colours 0 and 1, from the old odd rows y - 1 and y + 1) and then the odd
// row y - 1 (colours 2 and 3, from the new even rows y - 2 and y), so each
// cell's update reads exactly the values of the colour-ordered sweep, with
// k_gs_pair9's FMA chains.  The residual of odd row y - 1 is formed at the
// same step; that of even row y takes its slots 0..5 there and slots 6..8
// at the next step (k_resnorm's order).  The pass reads `in` and writes
// every row to `out`.  A wave owns 60 strips (lanes 2..61) and updates the
// two strips on either side too, storing nothing: the odd rows read the new
// even rows one cell beyond the owned range, and a halo strip's value there
// is right only when its own outer neighbour strip was updated as well.  A
// tile owns rows [y0, y1) with y0 even and updates again, without storing,
// the even rows y0 - 2 and y1 (and the odd row y0 - 1) that its own rows and
// residuals read.
constexpr int kSweepOwn = kWave - 4;

template <class Op, bool kRes>
__global__ __launch_bounds__(kBlock) void k_gs_sweep9(Op A, const double *__restrict__ b,
                                                      const double *__restrict__ in,
                                                      double *__restrict__ out, int mh,
                                                      double *part) {
    static_assert(Op::V == 2 && Op::NB == 9, "nine-point strips of two cells");
    constexpr int V = 2;
    using Unit = typename Op::Unit;
    const int lane = threadIdx.x % kWave;
    const int nx = A.nx, ny = A.ny;
    const int64_t upr = nx / V;
    const int64_t strips = (upr + kSweepOwn - 1) / kSweepOwn;
    const int64_t tiles = strips * (int64_t)((ny + mh - 1) / mh);
    double v[2] = {0.0, 0.0};
    for (int64_t t = (int64_t)logical_block() * kWaves + threadIdx.x / kWave; t < tiles;
         t += (int64_t)gridDim.x * kWaves) {
        const int64_t strip = t % strips, seg = t / strips;
        const int64_t xr = strip * kSweepOwn + lane - 2;
        const bool active = xr >= 0 && xr < upr;
        const bool owner = active && lane >= 2 && lane < 2 + kSweepOwn;
        const int xu = (int)(xr < 0 ? 0 : (xr >= upr ? upr - 1 : xr));
        const int x0 = xu * V;
        const int y0 = (int)seg * mh, y1 = min(ny, y0 + mh);
        const int ylast = (y1 + 1) & ~1;   // the first even row at or above y1
        auto old_row = [&](int y, double (&o)[V + 2]) {
            const int64_t sr = (int64_t)min(max(y, 0), ny - 1) * nx + x0;
            row_load<double, V>(in, sr, sr, x0, nx, y >= 0 && y < ny, true, o);
        };
        // one row's update: colour c0 = 2 (y mod 2) from old values, then
        // c0 + 1 with the new c0 values of its row; z rows s (y - 1), c (y,
        // old), n (y + 1) as the colour-ordered sweep sees them
        auto update = [&](const Unit &U, const double (&bb)[V], const double (&zs)[V + 2],
                          const double (&zc)[V + 2], const double (&zn)[V + 2],
                          double (&f)[V + 2]) {
            double nv[V];
#pragma unroll
            for (int k = 0; k < V; ++k) {
                double z[9];
                z[0] = zs[k]; z[1] = zs[k + 1]; z[2] = zs[k + 2];
                z[3] = zc[k]; z[4] = zc[k + 1]; z[5] = zc[k + 2];
                z[6] = zn[k]; z[7] = zn[k + 1]; z[8] = zn[k + 2];
                if (k == 1) {
                    z[3] = nv[0];
                    z[5] = __shfl_down(nv[0], 1, kWave);
                }
                double acc = bb[k], d = 1.0;
#pragma unroll
                for (int q = 0; q < 9; ++q) {
                    if (!A.valid(U, q, k)) continue;
                    if (q == Op::kC) d = U.a[q][k];
                    else acc = fma(-U.a[q][k], z[q], acc);
                }
                nv[k] = acc / d;
            }
            f[0] = __shfl_up(nv[1], 1, kWave);
            f[1] = nv[0];
            f[2] = nv[1];
            f[3] = __shfl_down(nv[0], 1, kWave);
        };
        double om1[V + 2], n2[V + 2], accp[V] = {0.0, 0.0};
        old_row(y0 - 3, om1);
#pragma unroll
        for (int k = 0; k < V + 2; ++k) n2[k] = 0.0;
        // the faces (N, NE, NW) of the even row of the previous step: the
        // south faces of this step's odd row, kept in registers (a step
        // later they are no longer in the cache); the even row's own south
        // faces are the odd row's arrays of the same step
        typename Op::South Sp{};
        for (int y = y0 - 2; y <= ylast; y += 2) {
            const bool real_e = y >= 0 && y < ny, real_o = y - 1 >= 0 && y - 1 < ny;
            double o0[V + 2], op1[V + 2];
            old_row(y, o0);
            old_row(y + 1, op1);
            // even row y
            Unit Ue;
            Ue.x0 = x0;
            Ue.y = y;
            double be[V] = {0.0, 0.0}, f0[V + 2];
            typename Op::South Se{};
            if (real_e) {
                A.geom_walk(Ue, (int64_t)y * upr + xu, xu, y);
                A.south_init(Se, Ue);
                A.load_row(Ue, Se);
                vld<double, V>(b + Ue.i0, be);
                update(Ue, be, om1, o0, op1, f0);
            } else {
#pragma unroll
                for (int k = 0; k < V + 2; ++k) f0[k] = 0.0;
            }
            if (owner && real_e && y >= y0 && y < y1) vst<double, V>(out + Ue.i0, {f0[1], f0[2]});
            if (y > y0 - 2) {
                // odd row y-1
                Unit Uo;
                Uo.x0 = x0;
                Uo.y = y - 1;
                double bo[V] = {0.0, 0.0}, f1[V + 2];
                double nw_x0 = 0.0, ne_x2 = 0.0;   // row y-2's NW at x0, NE at x0 + 2
                if (real_o) {
                    // row y-2 (even, >= 0 as y-1 is an odd row) was the
                    // previous step's even row
                    typename Op::South S = Sp;
                    A.geom_walk(Uo, (int64_t)(y - 1) * upr + xu, xu, y - 1);
                    nw_x0 = S.nw[0];
                    ne_x2 = S.ne[2];
                    A.load_row(Uo, S);
                    vld<double, V>(b + Uo.i0, bo);
                    update(Uo, bo, n2, om1, f0, f1);
                } else {
#pragma unroll
                    for (int k = 0; k < V + 2; ++k) f1[k] = 0.0;
                }
                if (owner && real_o && y - 1 >= y0 && y - 1 < y1)
                    vst<double, V>(out + Uo.i0, {f1[1], f1[2]});
                if (kRes && owner) {
                    // even row y-2: slots 6..8 (its NW, N, NE: the south
                    // faces of row y-1) over the new row y-1
                    if (y - 2 >= y0 && y - 2 < y1) {
                        Unit Ug;
                        Ug.x0 = x0;
                        Ug.y = y - 2;
                        const double a6[V] = {nw_x0, Uo.a[2][0]};
                        const double a7[V] = {Uo.a[1][0], Uo.a[1][1]};
                        const double a8[V] = {Uo.a[0][1], ne_x2};
#pragma unroll
                        for (int k = 0; k < V; ++k) {
                            double acc = accp[k];
                            if (real_o && A.valid(Ug, 6, k)) acc = fma(-a6[k], f1[k], acc);
                            if (real_o && A.valid(Ug, 7, k)) acc = fma(-a7[k], f1[k + 1], acc);
                            if (real_o && A.valid(Ug, 8, k)) acc = fma(-a8[k], f1[k + 2], acc);
                            v[0] += acc * acc;
                            const double m = fabs(acc);
                            v[1] = m > v[1] ? m : v[1];
                        }
                    }
                    // odd row y-1, whole
                    if (real_o && y - 1 >= y0 && y - 1 < y1) {
#pragma unroll
                        for (int k = 0; k < V; ++k) {
                            double z[9];
                            z[0] = n2[k]; z[1] = n2[k + 1]; z[2] = n2[k + 2];
                            z[3] = f1[k]; z[4] = f1[k + 1]; z[5] = f1[k + 2];
                            z[6] = f0[k]; z[7] = f0[k + 1]; z[8] = f0[k + 2];
                            double acc = bo[k];
#pragma unroll
                            for (int q = 0; q < 9; ++q)
                                if (A.valid(Uo, q, k)) acc = fma(-Uo.a[q][k], z[q], acc);
                            v[0] += acc * acc;
                            const double m = fabs(acc);
                            v[1] = m > v[1] ? m : v[1];
                        }
                    }
                    // even row y: slots 0..5 over the new rows y-1 and y
                    if (real_e) {
#pragma unroll
                        for (int k = 0; k < V; ++k) {
                            double z[6];
                            z[0] = f1[k]; z[1] = f1[k + 1]; z[2] = f1[k + 2];
                            z[3] = f0[k]; z[4] = f0[k + 1]; z[5] = f0[k + 2];
                            double acc = be[k];
#pragma unroll
                            for (int q = 0; q < 6; ++q)
                                if (A.valid(Ue, q, k)) acc = fma(-Ue.a[q][k], z[q], acc);
                            accp[k] = acc;
                        }
                    }
                }
            }
#pragma unroll
            for (int k = 0; k < V + 2; ++k) {
                om1[k] = op1[k];
                n2[k] = f0[k];
            }
            Sp = Se;
        }
    }
    if (kRes) write_partials<double, 2>(v, Ops<2u>(), part);
}

// ---------------------------------------------------------------------------
// single-synchronisation PCG (Jacobi or none): one kernel per iteration
// ---------------------------------------------------------------------------
// The recurrences of Chronopoulos and Gear: w_j = A z_j, and one combined
// reduction gamma_j = r_j.z_j, delta_j = w_j.z_j (plus rho_j = r_j.r_j for
// the stopping test) per iteration; beta_j = gamma_j / gamma_{j-1},
// alpha_j = gamma_j / (delta_j - beta_j gamma_j / alpha_{j-1}),
// p_j = z_j + beta_j p_{j-1}, s_j = w_j + beta_j s_{j-1} (= A p_j),
// x += alpha_j p_j, r_{j+1} = r_j - alpha_j s_j.  In exact arithmetic these
// are the iterates of the standard PCG.  With a pointwise preconditioner the
// next z is known at every neighbour, so w_{j+1} = A z_{j+1} is formed in
// the same pass: one launch and one reduction per iteration.  With Jacobi
// (M = diag) the stored vectors are scaled by M^-1: z_j = M^-1 r_j,
// M^-1 w_j and M^-1 s_j, so that z_{j+1} = z_j - alpha_j M^-1 s_j at a
// neighbour needs three gathered values and no division, and the own row
// forms r_{j+1} = diag z_{j+1} for the partials.  The buffers are
// double-buffered by iteration parity (neighbours read the old values); p
// and x are own-only.

// r_0 = rhs - A x (or rhs when x = 0); with the Jacobi preconditioner the
// kernel stores z_0 = r_0 / diag instead (the iteration keeps z, A z / diag
// and A p / diag in place of r, w and s)
template <class Op, int kPc>
__global__ __launch_bounds__(kBlock) void k_cg_init1(Op A, const typename Op::real *__restrict__ rhs,
                                                     const typename Op::real *__restrict__ x,
                                                     typename Op::real *__restrict__ r, int x_zero,
                                                     Scalars *sc) {
    using real = typename Op::real;
    constexpr int V = Op::V, NB = Op::NB;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        sc->pcg.done = 0;
        sc->pcg.status = kStOk;
        sc->pcg.it = 0;
    }
    for (auto W = walk<1>(A); W.valid(); W.advance()) {
        typename Op::Unit U;
        real rr[V];
        if (x_zero) {
            if (kPc == 1) W.load(A, U);   // the diagonal
            else W.geom(A, U);
            A.own(U, rhs, rr);
        } else {
            W.load(A, U);
            real xv[NB][V], bb[V];
            W.template gather<0>(A, U, x, xv);
            A.own(U, rhs, bb);
#pragma unroll
            for (int k = 0; k < V; ++k) {
                real acc = bb[k];
#pragma unroll
                for (int q = 0; q < NB; ++q)
                    if (A.valid(U, q, k)) acc = fma(-U.a[q][k], xv[q][k], acc);
                rr[k] = acc;
            }
        }
        if (kPc == 1) {
            real dd[V];
            diag_of(A, U, dd);
#pragma unroll
            for (int k = 0; k < V; ++k) rr[k] = rr[k] / dd[k];
        }
        A.put(U, r, rr);
    }
}

// w_0 = A z_0; partials gamma_0 = r_0.z_0, delta_0 = w_0.z_0, rho_0 = r_0.r_0.
// Jacobi: the input holds z_0 and the kernel stores w_0 / diag, with
// r_0 = diag z_0 for the partials; none: z_0 = r_0.
template <class Op, int kPc>
__global__ __launch_bounds__(kBlock) void k_cg_init2(Op A, const typename Op::real *__restrict__ r,
                                                     typename Op::real *__restrict__ w,
                                                     typename Op::real *part) {
    using real = typename Op::real;
    constexpr int V = Op::V, NB = Op::NB;
    real v[3] = {real(0), real(0), real(0)};
    for (auto W = walk<1>(A); W.valid(); W.advance()) {
        typename Op::Unit U;
        W.load(A, U);
        real zv[NB][V], ro[V], zo[V], wo[V], dd[V];
        W.template gather<0>(A, U, r, zv);
        own_of(A, U, zv, r, zo);
        if (kPc == 1) {
            diag_of(A, U, dd);
#pragma unroll
            for (int k = 0; k < V; ++k) ro[k] = dd[k] * zo[k];
        } else {
#pragma unroll
            for (int k = 0; k < V; ++k) ro[k] = zo[k];
        }
#pragma unroll
        for (int k = 0; k < V; ++k) {
            real acc = real(0);
#pragma unroll
            for (int q = 0; q < NB; ++q)
                if (A.valid(U, q, k)) acc = fma(U.a[q][k], zv[q][k], acc);
            wo[k] = kPc == 1 ? acc / dd[k] : acc;
            v[0] += ro[k] * zo[k];
            v[1] += acc * zo[k];
            v[2] += ro[k] * ro[k];
        }
        A.put(U, w, wo);
    }
    write_partials<real, 3>(v, Ops<0u>(), part);
}

// Iteration j.  Prologue: gamma_j, delta_j, rho_j from the partials -> stop
// (criterion on rho_j, max_iter, non-finite) or alpha_j, beta_j (breakdown
// when the denominator is not positive).  Body: p_j, s_j, x_{j+1}, r_{j+1}
// for the own cells, z_{j+1} at every neighbour, w_{j+1} = A z_{j+1}, and
// the partials gamma_{j+1}, delta_{j+1}, rho_{j+1}.
template <class Op, int kPc>
__global__ __launch_bounds__(kBlock) void k_cg_iter(
    Op A, typename Op::real *__restrict__ x, typename Op::real *__restrict__ p,
    const typename Op::real *__restrict__ s_old, typename Op::real *__restrict__ s_new,
    const typename Op::real *__restrict__ r_cur, typename Op::real *__restrict__ r_next,
    const typename Op::real *__restrict__ w_cur, typename Op::real *__restrict__ w_next, int j,
    int max_iter, const double *tol_base, double tol_factor, Scalars *sc,
    const typename Op::real *part_in, typename Op::real *part_out) {
    using real = typename Op::real;
    constexpr int V = Op::V, NB = Op::NB;
    // The scalars of the previous iterations, the stop flag and the first
    // unit's coefficients are loaded before the partial fold so that their
    // latencies overlap (block 0 of this launch writes other parities and
    // fields only; a block that sees the flag set by this launch would stop
    // anyway).
    const int done = sc->pcg.done;
    const double tol_prev = sc->pcg.tol;
    const double gamma_prev = sc->cg_gamma[(j - 1) & 1], alpha_prev = sc->cg_alpha[(j - 1) & 1];
    const double tol_in = (j == 0 && tol_base) ? *tol_base : 0.0;
    auto W = walk<3>(A);
    typename Op::Unit U;
    if (W.valid()) W.load(A, U);
    real t[3];
    read_partials<real, 3>(part_in, gridDim.x, Ops<0u>(), t);
    if (done) return;
    const double rho = (double)t[2];
    double tol;
    if (j == 0) tol = tol_base ? tol_factor * tol_in : tol_factor * sqrt(rho);
    else tol = tol_prev;
    int stop = 0, status = kStOk;
    real alpha = real(0), beta = real(0);
    if (!(rho == rho) || rho > 1.7e308) {
        stop = 1;
        status = kStNonFinite;
    } else if (sqrt(rho) <= tol) {
        stop = 1;
    } else if (j >= max_iter) {
        stop = 1;
        status = kStNoConv;
    } else {
        const real gamma = t[0], delta = t[1];
        real den = delta;
        if (j > 0) {
            beta = gamma / (real)gamma_prev;
            den = delta - beta * gamma / (real)alpha_prev;
        }
        if (!(den > real(0))) {
            stop = 1;
            status = (den == den) ? kStBreakdown : kStNonFinite;
        } else {
            alpha = gamma / den;
        }
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        if (j == 0) {
            sc->pcg.tol = tol;
            sc->pcg.rr0 = rho;
        }
        sc->pcg.rr = rho;
        sc->cg_gamma[j & 1] = (double)t[0];
        sc->cg_alpha[j & 1] = (double)alpha;
        if (stop) {
            sc->pcg.done = 1;
            sc->pcg.status = status;
            sc->pcg.it = j;
        }
    }
    if (stop) return;
    real v[3] = {real(0), real(0), real(0)};
    for (bool first = true; W.valid(); W.advance(), first = false) {
        if (!first) W.load(A, U);
        real rv[NB][V], wv[NB][V], ro[V], wo[V], xo[V], po[V], so[V], dd[V];
        W.template gather<0>(A, U, r_cur, rv);
        W.template gather<1>(A, U, w_cur, wv);
        own_of(A, U, rv, r_cur, ro);
        own_of(A, U, wv, w_cur, wo);
        A.own(U, (const real *)x, xo);
        if (kPc == 1) diag_of(A, U, dd);
        if (j > 0) {
            real sv[NB][V];
            W.template gather<2>(A, U, s_old, sv);
            own_of(A, U, sv, s_old, so);
            A.own(U, (const real *)p, po);
#pragma unroll
            for (int q = 0; q < NB; ++q)
#pragma unroll
                for (int k = 0; k < V; ++k) wv[q][k] = fma(beta, sv[q][k], wv[q][k]);
        }
        // neighbours: s = w + beta s_old (in wv), then the next z: with
        // Jacobi z - alpha s in the scaled vectors, else r' = r - alpha s
#pragma unroll
        for (int q = 0; q < NB; ++q)
#pragma unroll
            for (int k = 0; k < V; ++k)
                rv[q][k] = A.valid(U, q, k) ? fma(-alpha, wv[q][k], rv[q][k]) : real(0);
        real sn[V], rn[V], wn[V];
#pragma unroll
        for (int k = 0; k < V; ++k) {
            const real zk = ro[k];   // z_j (Jacobi: the stored z; none: r_j)
            const real pk = j > 0 ? fma(beta, po[k], zk) : zk;
            const real sk = j > 0 ? fma(beta, so[k], wo[k]) : wo[k];
            po[k] = pk;
            sn[k] = sk;
            xo[k] = fma(alpha, pk, xo[k]);
            const real zn = fma(-alpha, sk, ro[k]);
            real acc = real(0);
#pragma unroll
            for (int q = 0; q < NB; ++q)
                if (A.valid(U, q, k)) acc = fma(U.a[q][k], rv[q][k], acc);
            const real rk = kPc == 1 ? dd[k] * zn : zn;   // r_{j+1}
            rn[k] = zn;
            wn[k] = kPc == 1 ? acc / dd[k] : acc;
            v[0] += rk * zn;
            v[1] += acc * zn;
            v[2] += rk * rk;
        }
        A.put(U, x, xo);
        A.put(U, p, po);
        A.put(U, s_new, sn);
        A.put(U, r_next, rn);
        A.put(U, w_next, wn);
    }
    write_partials<real, 3>(v, Ops<0u>(), part_out);
}

// r = rhs - A x in FP64 (stored if r != null); partials ||r||^2, max|r|.
template <class Op>
__global__ __launch_bounds__(kBlock) void k_resnorm(Op A, const double *__restrict__ rhs,
                                                    const double *__restrict__ x,
                                                    double *__restrict__ r, double *part) {
    constexpr int V = Op::V, NB = Op::NB;
    double v[2] = {0.0, 0.0};
    for (auto W = walk<1>(A); W.valid(); W.advance()) {
        typename Op::Unit U;
        W.load(A, U);
        double xv[NB][V], bb[V], out[V];
        W.template gather<0>(A, U, x, xv);
        A.own(U, rhs, bb);
#pragma unroll
        for (int k = 0; k < V; ++k) {
            double acc = bb[k];
#pragma unroll
            for (int q = 0; q < NB; ++q)
                if (A.valid(U, q, k)) acc = fma(-U.a[q][k], xv[q][k], acc);
            out[k] = acc;
            v[0] += acc * acc;
            const double m = fabs(acc);
            v[1] = m > v[1] ? m : v[1];
        }
        if (r) A.put(U, r, out);
    }
    write_partials<double, 2>(v, Ops<2u>(), part);
}

// keep the outcome of a PCG run whose result the host reads later
__global__ void k_save_pcg(Scalars *sc, int scope) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        sc->saved_it[scope] = sc->pcg.it;
        sc->saved_status[scope] = sc->pcg.done ? sc->pcg.status : kStNoConv;
    }
}

// one block: fold the residual partials; done when ||r|| <= tol_factor * *tol_base
__global__ __launch_bounds__(kBlock) void k_fin_res(const double *part, int gprod,
                                                    const double *tol_base, double tol_factor,
                                                    Scalars *sc) {
    double tot[2];
    read_partials<double, 2>(part, gprod, Ops<2u>(), tot);
    if (threadIdx.x == 0) {
        ResState &s = sc->res;
        s.rr = tot[0];
        s.rmax = tot[1];
        s.tol = tol_factor * *tol_base;
        s.status = (tot[0] == tot[0]) ? kStOk : kStNonFinite;
        s.done = (s.status != kStOk || sqrt(tot[0]) <= s.tol) ? 1 : 0;
    }
}

// ||v||^2 partials, then one block folds them into *out = ||v||_2
__global__ __launch_bounds__(kBlock) void k_norm2(const double *__restrict__ v, int64_t n,
                                                  int64_t chunk, double *part) {
    const Chunk c = my_chunk(n, chunk);
    double a[1] = {0.0};
    for (int64_t i = c.begin + threadIdx.x; i < c.end; i += kBlock) a[0] += v[i] * v[i];
    write_partials<double, 1>(a, Ops<0u>(), part);
}

// ||a - b||^2 partials (chunked, like k_norm2)
__global__ __launch_bounds__(kBlock) void k_norm2_diff(const double *__restrict__ a,
                                                       const double *__restrict__ b, int64_t n,
                                                       int64_t chunk, double *part) {
    const Chunk c = my_chunk(n, chunk);
    double s[1] = {0.0};
    for (int64_t i = c.begin + threadIdx.x; i < c.end; i += kBlock) {
        const double d = a[i] - b[i];
        s[0] += d * d;
    }
    write_partials<double, 1>(s, Ops<0u>(), part);
}
__global__ __launch_bounds__(kBlock) void k_fin_norm(const double *part, int gprod, double *out) {
    double tot[1];
    read_partials<double, 1>(part, gprod, Ops<0u>(), tot);
    if (threadIdx.x == 0) *out = sqrt(tot[0]);
}

// ---------------------------------------------------------------------------
// mixed precision refinement helpers
// ---------------------------------------------------------------------------
// r32 = (float)(r / s) with s = max|r| (keeps the FP32 residual near 1 and
// clear of denormals); block 0 records s for the update.
// With guard set, a residual that already met the criterion or went
// non-finite (res.done) gives r32 = 0 and scale 0 instead: the inner solve
// then stops at its first test and the update leaves x as it is, so the host
// can enqueue a refinement step before it has read the residual.
__global__ __launch_bounds__(kBlock) void k_cast_scale(const double *__restrict__ r,
                                                       float *__restrict__ r32, int64_t n,
                                                       Scalars *sc, int guard) {
    const bool skip = guard && sc->res.done;
    const double s = sc->res.rmax > 0.0 ? sc->res.rmax : 1.0;
    if (blockIdx.x == 0 && threadIdx.x == 0) sc->scale = skip ? 0.0 : s;
    for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kBlock)
        r32[i] = skip ? 0.0f : (float)(r[i] / s);
}

// The start of one refinement step's inner solve with the single-sync PCG,
// in one pass: k_cast_scale's scaled right-hand side (same guard) written
// straight into r_0 (the inner solve starts from x = 0, so r_0 = rhs; with
// the Jacobi diagonal dg, z_0 = r_0 / dg as k_cg_init1 stores it), the
// inner x zeroed, and the PCG state reset as k_cg_init1 resets it.
__global__ __launch_bounds__(kBlock) void k_refine_start(const double *__restrict__ r,
                                                         const float *__restrict__ dg,
                                                         float *__restrict__ r0,
                                                         float *__restrict__ x32, int64_t n,
                                                         Scalars *sc, int guard) {
    const bool skip = guard && sc->res.done;
    const double s = sc->res.rmax > 0.0 ? sc->res.rmax : 1.0;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        sc->scale = skip ? 0.0 : s;
        sc->pcg.done = 0;
        sc->pcg.status = kStOk;
        sc->pcg.it = 0;
    }
    for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kBlock) {
        const float v = skip ? 0.0f : (float)(r[i] / s);
        r0[i] = dg ? v / dg[i] : v;
        x32[i] = 0.0f;
    }
}

// x += scale * d32: the FP64 update of one refinement step; skipped when the
// inner solve of that step broke down or went non-finite, so x keeps the
// last good iterate.  Also keeps the inner solve's outcome in
// saved_it / saved_status[scope] (k_save_pcg's work).  Nothing happens
// while the inner solve has not stopped (its stop flag unset): the host may
// enqueue the update behind the iterations it expects the solve to need,
// and enqueues more iterations and the update again if they were too few.
__global__ __launch_bounds__(kBlock) void k_axpy_scaled(double *__restrict__ x,
                                                        const float *__restrict__ d32,
                                                        int64_t n, Scalars *sc, int scope) {
    if (!sc->pcg.done) return;
    const int st = sc->pcg.status;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        sc->saved_it[scope] = sc->pcg.it;
        sc->saved_status[scope] = st;
    }
    if (st == kStBreakdown || st == kStNonFinite) return;
    const double s = sc->scale;
    for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kBlock)
        x[i] = fma(s, (double)d32[i], x[i]);
}

__global__ __launch_bounds__(kBlock) void k_cast(const double *__restrict__ a,
                                                 float *__restrict__ b, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kBlock)
        b[i] = (float)a[i];
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_fill(T *__restrict__ a, T v, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kBlock)
        a[i] = v;
}

// y = A x (measurement of the stencil SpMV on its own)
template <class Op>
__global__ __launch_bounds__(kBlock) void k_spmv(Op A, const typename Op::real *__restrict__ x,
                                                 typename Op::real *__restrict__ y) {
    using real = typename Op::real;
    constexpr int V = Op::V, NB = Op::NB;
    for (auto W = walk<1>(A); W.valid(); W.advance()) {
        typename Op::Unit U;
        W.load(A, U);
        real xv[NB][V], out[V];
        W.template gather<0>(A, U, x, xv);
#pragma unroll
        for (int k = 0; k < V; ++k) {
            real acc = real(0);
#pragma unroll
            for (int q = 0; q < NB; ++q)
                if (A.valid(U, q, k)) acc = fma(U.a[q][k], xv[q][k], acc);
            out[k] = acc;
        }
        A.put(U, y, out);
    }
}

// ---------------------------------------------------------------------------
// adjoint helpers: operator from log-conductivity and its derivative
// ---------------------------------------------------------------------------
__device__ __forceinline__ double harmonic(double kp, double kq) { return 2.0 * kp * kq / (kp + kq); }

// one thread per cell: the cell's own forward faces plus the diagonal sum of
// all its faces (each face value recomputed by both cells: no atomics)
template <int kDim>
__global__ __launch_bounds__(kBlock) void k_assemble_logk(int nx, int ny, int nz, double inv_dt,
                                                          const double *__restrict__ logk,
                                                          double *__restrict__ coef) {
    const int64_t n = (int64_t)nx * ny * nz, pl = (int64_t)nx * ny;
    for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kBlock) {
        const int z = (int)(i / pl);
        const int rr = (int)(i - (int64_t)z * pl);
        const int y = rr / nx, x = rr - y * nx;
        const double kp = exp(logk[i]);
        double tw = 0, te = 0, ts = 0, tn = 0, td = 0, tu = 0;
        if (x > 0) tw = harmonic(exp(logk[i - 1]), kp);
        if (x < nx - 1) te = harmonic(kp, exp(logk[i + 1]));
        if (y > 0) ts = harmonic(exp(logk[i - nx]), kp);
        if (y < ny - 1) tn = harmonic(kp, exp(logk[i + nx]));
        if (kDim == 3) {
            if (z > 0) td = harmonic(exp(logk[i - pl]), kp);
            if (z < nz - 1) tu = harmonic(kp, exp(logk[i + pl]));
        }
        double d = inv_dt;
        d += tw; d += te; d += ts; d += tn;
        if (kDim == 3) { d += td; d += tu; }
        coef[i] = d;
        coef[n + i] = -te;
        coef[2 * n + i] = -tn;
        if (kDim == 3) coef[3 * n + i] = -tu;
    }
}

// Picard system of the 2-D heat-conduction test (Section 3.1, eq.
// picard-equs): cell-centred finite volumes scaled by h^2, k = T_lin^power,
// interior faces take the arithmetic mean (k_P + k_Q) / 2 (the harmonic mean
// would close the faces into the cold region, k(1e-4) = 1e-14, and the front
// could not advance), Dirichlet faces at x = 0 / x = 1 half a cell away
// (transmissibility 2 * mean(k_b, k_P), rhs gains it times T_b), zero flux
// in y.  One thread per cell; diagonal sums in the order 1/dt, west, east,
// south, north.
__device__ __forceinline__ double kpow(double t, double power) { return exp(power * log(t)); }
__device__ __forceinline__ double face_mean(double kp, double kq) { return 0.5 * (kp + kq); }
__global__ __launch_bounds__(kBlock) void k_assemble_heat(int nx, int ny, double inv_dt, double power,
                                                          double tl, double tr,
                                                          const double *__restrict__ tlin,
                                                          const double *__restrict__ told,
                                                          double *__restrict__ coef,
                                                          double *__restrict__ b) {
    const int64_t n = (int64_t)nx * ny;
    const double kl = kpow(tl, power), kr = kpow(tr, power);
    for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kBlock) {
        const int y = (int)(i / nx), x = (int)(i - (int64_t)y * nx);
        const double kp = kpow(tlin[i], power);
        const double tw = x > 0 ? face_mean(kpow(tlin[i - 1], power), kp) : 2.0 * face_mean(kl, kp);
        const double te = x < nx - 1 ? face_mean(kp, kpow(tlin[i + 1], power)) : 2.0 * face_mean(kp, kr);
        const double ts = y > 0 ? face_mean(kpow(tlin[i - nx], power), kp) : 0.0;
        const double tn = y < ny - 1 ? face_mean(kp, kpow(tlin[i + nx], power)) : 0.0;
        double d = inv_dt;
        d += tw;
        d += te;
        d += ts;
        d += tn;
        coef[i] = d;
        coef[n + i] = x < nx - 1 ? -te : 0.0;
        coef[2 * n + i] = y < ny - 1 ? -tn : 0.0;
        double r = told[i] * inv_dt;
        if (x == 0) r += tw * tl;
        if (x == nx - 1) r += te * tr;
        b[i] = r;
    }
}

template <int kDim>
__global__ __launch_bounds__(kBlock) void k_grad_logk(int nx, int ny, int nz,
                                                      const double *__restrict__ logk,
                                                      const double *__restrict__ xv,
                                                      const double *__restrict__ lam,
                                                      double *__restrict__ grad) {
    const int64_t n = (int64_t)nx * ny * nz, pl = (int64_t)nx * ny;
    for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kBlock) {
        const int z = (int)(i / pl);
        const int rr = (int)(i - (int64_t)z * pl);
        const int y = rr / nx, x = rr - y * nx;
        const double kp = exp(logk[i]), xp = xv[i], lp = lam[i];
        double s = 0.0;
        auto face = [&](int64_t j) {
            const double kq = exp(logk[j]);
            const double t = harmonic(kp, kq);
            const double dtdl = t * kq / (kp + kq);
            s += dtdl * (xp - xv[j]) * (lp - lam[j]);
        };
        if (kDim == 3 && z > 0) face(i - pl);
        if (y > 0) face(i - nx);
        if (x > 0) face(i - 1);
        if (x < nx - 1) face(i + 1);
        if (y < ny - 1) face(i + nx);
        if (kDim == 3 && z < nz - 1) face(i + pl);
        grad[i] = -s;
    }
}

}  // namespace lcs
