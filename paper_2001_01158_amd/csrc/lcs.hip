// Host runtime and C ABI of the local character-based solver (see lcs.h).
//
// Every step of the method runs in the kernels of lcs_kernels.h; the host
// only sizes launches, orders them on the caller's stream and reads a few
// scalars (K, convergence flags) back through pinned memory.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <functional>
#include <limits>
#include <mutex>
#include <string>
#include <type_traits>
#include <vector>

#include "lcs.h"
#include "lcs_kernels.h"
#include "lcs_batched.h"
#include "lcs_gmres.h"
#include "lcs_csr.h"

using namespace lcs;

namespace {

thread_local std::string g_err;

lcs_status fail(lcs_status s, const std::string &msg) {
    g_err = msg;
    return s;
}

#define HIP_TRY(expr)                                                                  \
    do {                                                                               \
        hipError_t e_ = (expr);                                                        \
        if (e_ != hipSuccess)                                                          \
            return fail(LCS_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

#define LCS_TRY(expr)                \
    do {                             \
        lcs_status s_ = (expr);      \
        if (s_ != LCS_OK) return s_; \
    } while (0)

#define LAUNCH_CHECK()                                                            \
    do {                                                                          \
        hipError_t e_ = hipGetLastError();                                        \
        if (e_ != hipSuccess)                                                     \
            return fail(LCS_EHIP, std::string("launch: ") + hipGetErrorString(e_)); \
    } while (0)

int n_arrays(int kind) {
    return kind == LCS_STENCIL5_2D ? 3 : kind == LCS_STENCIL9_2D ? 5 : kind == LCS_STENCIL9N_2D ? 9 : 4;
}
int n_colours(int kind) { return kind == LCS_STENCIL9_2D || kind == LCS_STENCIL9N_2D ? 4 : 2; }
// solves by GMRES(m): the non-symmetric stencil and non-symmetric CSR input
bool uses_gmres(const lcs_matrix *A) {
    return A->kind == LCS_STENCIL9N_2D || (A->kind == LCS_CSR && A->csr_nonsym);
}
// colours of the Gauss-Seidel sweeps; 0 for a general sparse matrix given
// without a colouring (no sweeps)
int colours_of(const lcs_matrix *A) {
    return A->kind == LCS_CSR ? (A->colour ? A->n_colours : 0) : n_colours(A->kind);
}

// Largest |j - i| between a grid row i and a stencil neighbour j (the
// index distance, in grid order, that a member of a restricted row can lie
// from the row); unbounded for general sparse input.
int64_t stencil_reach(const lcs_matrix *A) {
    switch (A->kind) {
    case LCS_STENCIL5_2D: return A->nx;
    case LCS_STENCIL9_2D:
    case LCS_STENCIL9N_2D: return (int64_t)A->nx + 1;
    case LCS_STENCIL7_3D: return (int64_t)A->nx * A->ny;
    default: return std::numeric_limits<int64_t>::max();
    }
}

struct Launch {
    int grid;
    int64_t chunk;
};

// Chunked grid: at most kMaxGrid blocks (a multiple of 8 once large enough,
// for the XCD remap), each owning `chunk` consecutive rows.
// Chunked grid of up to `cap` blocks (<= kSlotElems for kernels that write
// one partial per block), for per-row kernels whose rows are latency-bound
// chains of dependent loads: more blocks, fewer rows per thread.
Launch dims_wide(int64_t n, int cap) {
    int64_t g = (n + kBlock - 1) / kBlock;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    if (g >= 64) g = (g + kXcds - 1) / kXcds * kXcds;
    int64_t chunk = (n + g - 1) / g;
    if (chunk < 1) chunk = 1;
    return {(int)g, chunk};
}

Launch dims_for(int64_t n) {
    int64_t g = (n + kBlock - 1) / kBlock;
    if (g < 1) g = 1;
    if (g > kMaxGrid) g = kMaxGrid;
    if (g >= 64) g = (g + kXcds - 1) / kXcds * kXcds;
    int64_t chunk = (n + g - 1) / g;
    if (chunk < 1) chunk = 1;
    return {(int)g, chunk};
}

int flat_grid(int64_t n) {
    int64_t g = (n + kBlock - 1) / kBlock;
    if (g < 1) g = 1;
    if (g > 8 * kMaxGrid) g = 8 * kMaxGrid;
    return (int)g;
}

// Grid of the band kernels: a multiple of 8 (one band per XCD).  Kernels
// whose partials the next kernel folds keep at most kMaxGrid blocks (each
// consumer block reads them all); the others may use more.
int band_grid(int64_t units, int cap) {
    int64_t g = (units + kBlock - 1) / kBlock;
    g = (g + kXcds - 1) / kXcds * kXcds;
    if (g < kXcds) g = kXcds;
    if (g > cap) g = cap;
    return (int)g;
}
constexpr int kRedGrid = 512;     // reducing band kernels
constexpr int kStreamGrid = 4096; // non-reducing band kernels

// Grid of a unit-operator kernel: one wave per row-marching tile for the 2-D
// stencils (waves loop over tiles beyond the cap), else the band grid.  The
// reducing kernels on ELL rows (restricted systems, general sparse input)
// take up to kMaxGrid blocks: their rows are gathers whose latency more
// waves hide, and the fold of 1024 partials costs one round of loads.
template <class Op>
int grid_for(const Op &A, int cap) {
    if constexpr (Op::kMarch) {
        int64_t g = (A.tiles() + kWaves - 1) / kWaves;
        g = (g + kXcds - 1) / kXcds * kXcds;
        g = std::max<int64_t>(kXcds, std::min<int64_t>(g, cap));
        return (int)g;
    } else {
        return band_grid(A.units(), cap == kRedGrid ? kMaxGrid : cap);
    }
}

// Compaction tiling: tiles of kTile stamps, at most kMaxGrid blocks.
struct Tiling {
    int grid;
    int64_t ntiles, tiles_per_block, npad;
};
Tiling tiling_for(int64_t n) {
    Tiling t;
    t.ntiles = (n + kTile - 1) / kTile;
    if (t.ntiles < 1) t.ntiles = 1;
    int64_t g = std::min<int64_t>(t.ntiles, kMaxGrid);
    t.tiles_per_block = (t.ntiles + g - 1) / g;
    t.grid = (int)((t.ntiles + t.tiles_per_block - 1) / t.tiles_per_block);
    t.npad = t.ntiles * kTile;
    return t;
}

enum BufId {
    B_SCORE, B_R, B_Z, B_P0, B_P1, B_Q, B_RHSL, B_DL, B_RES, B_STAMP, B_INV, B_IDX, B_BLOCKOFF,
    B_ROWLEN, B_RP, B_COL, B_VAL, B_VAL32, B_DG, B_DG32, B_CLR, B_R32, B_D32, B_RI32, B_Z32,
    B_P32A, B_P32B, B_Q32, B_COEF32, B_CSRCOL, B_CSRVAL, B_W0, B_W1, B_S0, B_S1, B_W32A, B_W32B,
    B_S32A, B_S32B, B_BWS, B_BSTAMP, B_BIDX, B_BOUT, B_GMV, B_GMW0, B_GMW1, B_GMP0,
    B_GMPN, B_GMS, B_BGMV, B_ACOL, B_AVAL, B_ACLR, B_AFLAGS, B_GSX, B_IDXB, B_CBLK, B_NUM
};

}  // namespace

struct lcs_ctx {
    int device = 0;
    Scalars *dsc = nullptr;    // device state
    Scalars *hsc = nullptr;    // pinned host copy
    int32_t *hdone = nullptr;  // pinned: the GMRES done flag
    PcgState *hpcg = nullptr;  // pinned: two slots of the PCG state for asynchronous checks
    double *partials = nullptr;
    void *buf[B_NUM] = {};
    size_t cap[B_NUM] = {};
    // caller-owned workspace (lcs_create_with_workspace): the state, the
    // partials and every buffer are carved from it at offsets planned at the
    // start of each call; null: the context owns grow-only buffers
    char *ws = nullptr;
    size_t ws_bytes = 0;
    size_t ws_off[B_NUM] = {};
    size_t ws_len[B_NUM] = {};
    hipEvent_t ev[5] = {};
    hipEvent_t chk[2] = {};
    hipEvent_t done_ev = nullptr;   // recorded by wait_for (null: block instead)
    // rows of the restricted system blocked by colour during a local solve:
    // colour q in [start[q], start[q + 1]); n = 0 when not blocked
    struct {
        int n = 0;
        int64_t start[kMaxBlkColours + 1] = {};
    } cblk;
    // iterations of the previous global (0) / local (1) PCG, by refinement
    // step (mixed precision) or restart (FP64), for sizing the first chunk
    int last_its[2][4] = {};
    int cur_outer = 0;              // refinement step of the PCG being run
    // optional kernel timing (HIP events around one kernel class)
    int prof_what = 0;              // LCS_TIME_* or 0
    std::vector<hipEvent_t> prof_ev;
    size_t prof_used = 0;
    double prof_ms = 0.0;
    int64_t prof_launches = 0;
    // restricted systems reordered by colour under RB-SGS (lcs_set_colour_blocking)
    int colour_blocks = 1;
    // 16-bit column offsets in restricted systems where they fit
    // (lcs_set_short_columns)
    int short_cols = 1;
    // row-marching tiling of the 2-D stencil kernels (0 / -1: automatic)
    int march_rows = 0;
    int nontemporal = -1;
    // pinned host copy of the per-system results of a batched solve, read
    // back kBoutChunk systems at a time
    BatchOut *hbout = nullptr;
    // pinned host copy of the GMRES cycle state
    GmState *hgm = nullptr;
    // ELL copy of the general sparse matrix of the current call
    struct {
        int width = 0;         // 5, 7, 9, 16 or 64
        int64_t n = 0;
        int32_t *col = nullptr;
        double *val = nullptr;   // width x n values, then the diagonal
        uint8_t *clr = nullptr;
        // the matrix the copy was made from (valid after a successful check)
        bool valid = false;
        const void *rp = nullptr, *col_in = nullptr, *val_in = nullptr, *clr_in = nullptr;
        int64_t nnz = 0;
        int32_t ncol = 0;
    } ell;
};

namespace {

template <typename T>
lcs_status get_buf(lcs_ctx *c, BufId id, size_t count, T **out) {
    const size_t bytes = std::max<size_t>(count, 1) * sizeof(T);
    if (c->ws) {   // caller-owned workspace: the slot planned for this call
        if (c->ws_len[id] < bytes)
            return fail(LCS_EINVAL, "workspace plan holds " + std::to_string(c->ws_len[id]) +
                                        " bytes for buffer " + std::to_string((int)id) + ", " +
                                        std::to_string(bytes) + " requested");
        *out = reinterpret_cast<T *>(c->ws + c->ws_off[id]);
        return LCS_OK;
    }
    if (c->cap[id] < bytes) {
        // Slack for sequences whose K grows: an eighth on the first
        // allocation, half once a buffer has had to grow (each regrowth
        // synchronises the device and costs about a millisecond).
        const bool regrow = c->buf[id] != nullptr;
        if (c->buf[id]) {
            HIP_TRY(hipDeviceSynchronize());  // the old buffer may still be in use
            HIP_TRY(hipFree(c->buf[id]));
        }
        c->buf[id] = nullptr;
        c->cap[id] = 0;
        const size_t want = bytes + (regrow ? bytes / 2 : bytes / 8);
        if (hipMalloc(&c->buf[id], want) != hipSuccess) {
            (void)hipGetLastError();
            return fail(LCS_ENOMEM, "device workspace allocation of " + std::to_string(want) +
                                        " bytes failed");
        }
        c->cap[id] = want;
    }
    *out = static_cast<T *>(c->buf[id]);
    return LCS_OK;
}

double *slot(lcs_ctx *c, int k) { return c->partials + (size_t)k * kSlotElems; }
template <typename real>
real *slot_as(lcs_ctx *c, int k) { return reinterpret_cast<real *>(slot(c, k)); }

// Wait for an event by polling it.  A blocking wait sleeps until an
// interrupt and resumes tens of microseconds after the GPU gets there; a
// solve waits on the host several times (each chunk check, each refinement
// step), so the poll, which resumes within a few microseconds, saves a
// visible share of a millisecond-scale solve.  After kSpinUs of polling the
// wait blocks.  Polling leaves hipErrorNotReady as the thread's last error,
// which is cleared so that later launch checks (ours or the caller's) do
// not see it.
constexpr double kSpinUs = 2000.0;

lcs_status spin_event(hipEvent_t e) {
    const auto t0 = std::chrono::steady_clock::now();
    hipError_t q = hipErrorNotReady;
    for (int k = 0; q == hipErrorNotReady; ++k) {
        q = hipEventQuery(e);
        if (q == hipErrorNotReady && (k & 63) == 63 &&
            std::chrono::duration<double, std::micro>(std::chrono::steady_clock::now() - t0).count() >
                kSpinUs)
            break;
    }
    if (hipPeekAtLastError() == hipErrorNotReady) (void)hipGetLastError();
    if (q == hipSuccess) return LCS_OK;
    if (q != hipErrorNotReady)
        return fail(LCS_EHIP, std::string("hipEventQuery: ") + hipGetErrorString(q));
    HIP_TRY(hipEventSynchronize(e));
    return LCS_OK;
}

// Wait until stream s has executed everything enqueued so far.
lcs_status wait_for(lcs_ctx *c, hipStream_t s) {
    if (!c->done_ev) {   // a context without events (the allocation-free path)
        HIP_TRY(hipStreamSynchronize(s));
        return LCS_OK;
    }
    HIP_TRY(hipEventRecord(c->done_ev, s));
    return spin_event(c->done_ev);
}

// Record done_ev on s, for a later wait_recorded (work enqueued before a
// wait, such as a refinement step's tail).
lcs_status record_done(lcs_ctx *c, hipStream_t s) {
    if (c->done_ev) HIP_TRY(hipEventRecord(c->done_ev, s));
    return LCS_OK;
}
lcs_status wait_recorded(lcs_ctx *c, hipStream_t s) {
    if (!c->done_ev) {
        HIP_TRY(hipStreamSynchronize(s));
        return LCS_OK;
    }
    return spin_event(c->done_ev);
}

lcs_status read_scalars(lcs_ctx *c, hipStream_t s) {
    HIP_TRY(hipMemcpyAsync(c->hsc, c->dsc, sizeof(Scalars), hipMemcpyDeviceToHost, s));
    return wait_for(c, s);
}

lcs_status check_matrix(const lcs_matrix *A) {
    if (!A) return fail(LCS_EINVAL, "matrix is NULL");
    if (A->kind < 0 || A->kind > 4) return fail(LCS_EINVAL, "unknown matrix kind");
    if (A->nx < 1 || A->ny < 1 || A->nz < 1) return fail(LCS_EINVAL, "grid sizes must be >= 1");
    if (A->kind == LCS_CSR) {
        if (A->ny != 1 || A->nz != 1) return fail(LCS_EINVAL, "a CSR matrix has nx = N, ny = nz = 1");
        if (A->nx >= (1 << 27)) return fail(LCS_EINVAL, "N must be < 2^27");
        if (!A->row_ptr || !A->col || !A->val) return fail(LCS_EINVAL, "row_ptr, col or val is NULL");
        if (A->nnz < 1 || A->nnz > (int64_t)kCsrMaxRow * A->nx)
            return fail(LCS_EINVAL, "nnz must be in 1 .. 64 N");
        if (A->colour && (A->n_colours < 1 || A->n_colours > 255))
            return fail(LCS_EINVAL, "n_colours must be 1..255 with a colouring");
        return LCS_OK;
    }
    if (A->kind != LCS_STENCIL7_3D && A->nz != 1) return fail(LCS_EINVAL, "2-D stencil needs nz = 1");
    const int64_t n = (int64_t)A->nx * A->ny * A->nz;
    if (n >= ((int64_t)1 << 31) / 16) return fail(LCS_EINVAL, "N must be < 2^27");
    if (!A->coef) return fail(LCS_EINVAL, "coef is NULL");
    return LCS_OK;
}

lcs_status check_options(const lcs_options *o, int kind) {
    if (!o) return fail(LCS_EINVAL, "options are NULL");
    if (!(o->eps > 0.0)) return fail(LCS_EINVAL, "eps must be > 0");
    if (o->max_iter < 0 || o->n_smooth < 0 || o->max_outer < 0)
        return fail(LCS_EINVAL, "negative iteration counts");
    if (o->precond < 0 || o->precond > 2) return fail(LCS_EINVAL, "unknown preconditioner");
    if (o->precision < 0 || o->precision > 1) return fail(LCS_EINVAL, "unknown precision");
    if (o->precond == LCS_PC_RBSGS && kind == LCS_STENCIL9N_2D)
        return fail(LCS_EINVAL, "symmetric Gauss-Seidel needs a symmetric operator");
    if (kind == LCS_STENCIL9N_2D) {
        if (o->precision != LCS_PREC_FP64)
            return fail(LCS_EINVAL, "the non-symmetric operator is solved by GMRES in FP64");
        if (o->restart < 1 || o->restart > kMaxRestart)
            return fail(LCS_EINVAL, "GMRES restart length must be 1..64");
    }
    return LCS_OK;
}

lcs_status check_options_for(const lcs_options *o, const lcs_matrix *A) {
    // non-symmetric CSR input follows the non-symmetric stencil's rules
    LCS_TRY(check_options(o, uses_gmres(A) ? (int)LCS_STENCIL9N_2D : A->kind));
    if (A->kind == LCS_CSR && o->precond == LCS_PC_RBSGS && !A->colour)
        return fail(LCS_EINVAL, "symmetric Gauss-Seidel on a CSR matrix needs its colouring");
    return LCS_OK;
}

lcs_status check_ptr(const void *p, const char *what) {
    if (!p) return fail(LCS_EINVAL, std::string(what) + " is NULL");
    return LCS_OK;
}

// ---------------------------------------------------------------------------
// caller-owned workspace: the layout of one call
// ---------------------------------------------------------------------------
// What a call may request from the workspace.  Each class requests the
// buffers listed in plan_sizes at most at their largest size (K = N).
enum What { kWhatPiece = 0, kWhatSpmv32, kWhatDomain, kWhatGather, kWhatSolve, kWhatBatch };
constexpr size_t kWsAlign = 256;
constexpr int kBoutChunk = 1024;   // batched results read back this many at a time

size_t align_up(size_t v) { return (v + kWsAlign - 1) / kWsAlign * kWsAlign; }

// the state and the reduction partials at the head of a workspace
size_t ws_head_bytes() {
    return align_up(sizeof(Scalars)) + align_up(sizeof(double) * kSlotElems * kPtSlots);
}

// slots of the restricted ELL matrix: the stencil's entries per row, or
// the widest ELL copy of general sparse input
int gather_width(const lcs_matrix *A) {
    switch (A->kind) {
    case LCS_STENCIL5_2D: return 5;
    case LCS_STENCIL7_3D: return 7;
    case LCS_CSR: return kCsrMaxRow;
    default: return 9;
    }
}

// Bytes of every buffer a call of class `what` on A with options o (NULL:
// the defaults) may request, at its largest; 0 for the buffers it never
// requests.  G: systems of a batched call.
void plan_sizes(const lcs_matrix *A, const lcs_options *o, int what, int64_t G,
                size_t len[B_NUM]) {
    for (int i = 0; i < B_NUM; ++i) len[i] = 0;
    lcs_options def;
    if (!o) {
        lcs_default_options(&def);
        o = &def;
    }
    const size_t n = (size_t)A->nx * A->ny * A->nz;
    const size_t d = sizeof(double), f = sizeof(float), i4 = sizeof(int32_t);
    const bool csr = A->kind == LCS_CSR;
    const bool mixed = o->precision == LCS_PREC_MIXED;
    if (csr) {   // the checked ELL copy of width <= 16 and its diagonal
        len[B_AFLAGS] = 2 * i4;
        len[B_ACOL] = (size_t)kCsrMaxRow * n * i4;
        len[B_AVAL] = (size_t)(kCsrMaxRow + 1) * n * d;
        len[B_ACLR] = n;
    }
    const bool want32 = what == kWhatSpmv32 || (what == kWhatSolve && mixed);
    if (want32 && (csr || !A->coef32))
        len[B_COEF32] = (csr ? (size_t)(kCsrMaxRow + 1) : (size_t)n_arrays(A->kind)) * n * f;
    const size_t W = (size_t)gather_width(A);
    const size_t blockoff = 2 * (size_t)kMaxGrid * i4;
    // the second buffer of the paired-colour sweeps of the nine-point stencil
    if (A->kind == LCS_STENCIL9_2D && (what == kWhatPiece || what == kWhatSolve))
        len[B_GSX] = n * d;
    if (what == kWhatDomain || what == kWhatSolve) {
        len[B_SCORE] = n * d;
        len[B_STAMP] = (size_t)tiling_for((int64_t)n).npad;
        len[B_INV] = n * i4;
        len[B_BLOCKOFF] = blockoff;
    }
    if (what == kWhatGather || what == kWhatSolve) {
        len[B_INV] = n * i4;
        len[B_COL] = W * n * i4;
        len[B_VAL] = W * n * d;
        len[B_DG] = n * d;
        len[B_CLR] = n;
        len[B_RHSL] = n * d;
        len[B_ROWLEN] = n * i4;
        len[B_BLOCKOFF] = blockoff;
    }
    if (what == kWhatSolve) {
        len[B_IDX] = n * i4;
        len[B_DL] = n * d;
        if (o->precond == LCS_PC_RBSGS) {   // the colour-blocked domain
            len[B_IDXB] = n * i4;
            len[B_CBLK] = (size_t)kMaxBlkColours * kMaxGrid * i4;
        }
        if (uses_gmres(A)) {
            const size_t m = (size_t)std::max(1, std::min(o->restart > 0 ? o->restart : 40, kMaxRestart));
            len[B_GMV] = (m + 1) * n * d;
            len[B_GMW0] = len[B_GMW1] = n * d;
            len[B_GMP0] = (size_t)kGmPartVals * kGmGrid * d;
            len[B_GMPN] = (size_t)kGmGrid * d;
            len[B_GMS] = sizeof(GmState);
        } else if (!mixed) {
            for (BufId b : {B_R, B_Z, B_P0, B_P1, B_Q, B_W0, B_W1, B_S0, B_S1}) len[b] = n * d;
        } else {
            len[B_VAL32] = W * n * f;
            len[B_DG32] = n * f;
            len[B_RES] = n * d;
            for (BufId b : {B_R32, B_D32, B_RI32, B_Z32, B_P32A, B_P32B, B_Q32, B_W32A, B_W32B,
                            B_S32A, B_S32B})
                len[b] = n * f;
        }
    }
    if (what == kWhatBatch) {
        const size_t g = (size_t)std::max<int64_t>(G, 1);
        len[B_BWS] = 4 * n * g * d;
        len[B_BSTAMP] = n * g;
        len[B_BIDX] = n * g * i4;
        len[B_BOUT] = g * sizeof(BatchOut);
        if (A->kind == LCS_STENCIL9N_2D)
            len[B_BGMV] = (size_t)(std::max(1, std::min(o->restart, kMaxRestart)) + 1) * n * g * d;
    }
}

// Offsets of the planned buffers after the head: the ELL copy of general
// sparse input first (its place depends on N alone, so a copy kept for
// csr_reuse stays where it is), then the others in BufId order.  Returns
// the total bytes.
size_t plan_offsets(const size_t len[B_NUM], size_t off[B_NUM]) {
    size_t at = ws_head_bytes();
    const BufId first[] = {B_AFLAGS, B_ACOL, B_AVAL, B_ACLR};
    for (BufId b : first) {
        off[b] = at;
        at += align_up(len[b]);
    }
    for (int i = 0; i < B_NUM; ++i) {
        if (i == B_AFLAGS || i == B_ACOL || i == B_AVAL || i == B_ACLR) continue;
        off[i] = at;
        at += align_up(len[i]);
    }
    return at;
}

size_t plan_total(const lcs_matrix *A, const lcs_options *o, int what, int64_t G) {
    size_t len[B_NUM], off[B_NUM];
    plan_sizes(A, o, what, G, len);
    return plan_offsets(len, off);
}

// At the start of a call on a context with a caller-owned workspace: lay out
// the buffers this call may use, or fail with LCS_EINVAL before any work if
// the workspace is too small.  A call on another matrix may overwrite a kept
// ELL copy, so only general sparse input keeps it.
lcs_status plan_call(lcs_ctx *c, const lcs_matrix *A, const lcs_options *o, int what,
                     int64_t G = 0) {
    if (!c->ws) return LCS_OK;
    plan_sizes(A, o, what, G, c->ws_len);
    const size_t total = plan_offsets(c->ws_len, c->ws_off);
    if (A->kind != LCS_CSR) c->ell.valid = false;
    if (total > c->ws_bytes)
        return fail(LCS_EINVAL, "workspace of " + std::to_string(c->ws_bytes) +
                                    " bytes is smaller than the " + std::to_string(total) +
                                    " bytes this call needs (lcs_workspace_bytes)");
    return LCS_OK;
}

// ---------------------------------------------------------------------------
// operators from the C description
// ---------------------------------------------------------------------------
// Scalar row operators (marking rounds, gather) and unit operators for the
// grid-sized kernels.  Vector width: FP64 strips of 2, FP32 strips of 4 when
// nx is a multiple of 4 and every pointer is 16-byte aligned, else 1.
template <typename real>
Stencil5<real> sop5(const lcs_matrix *A, const real *c) {
    const int64_t n = (int64_t)A->nx * A->ny;
    return {c, c + n, c + 2 * n, A->nx, A->ny, n};
}
template <typename real>
Stencil9<real> sop9(const lcs_matrix *A, const real *c) {
    const int64_t n = (int64_t)A->nx * A->ny;
    return {c, c + n, c + 2 * n, c + 3 * n, c + 4 * n, A->nx, A->ny, n};
}
template <typename real>
Stencil9N<real> sop9n(const lcs_matrix *A, const real *c) {
    return {c, A->nx, A->ny, (int64_t)A->nx * A->ny};
}
template <typename real>
U9N<real, 1> uop9n(const lcs_matrix *A, const real *c) {
    return {c, A->nx, A->ny, (int64_t)A->nx * A->ny};
}
template <typename real>
Stencil7<real> sop7(const lcs_matrix *A, const real *c) {
    const int64_t n = (int64_t)A->nx * A->ny * A->nz;
    return {c, c + n, c + 2 * n, c + 3 * n, A->nx, A->ny, A->nz, n};
}
// Row-marching tiles of the 2-D unit operators: about 2048 tiles (8 waves
// per CU) of at most 32 rows.  The own-cell coefficient arrays are read with
// non-temporal loads once a pass streams more than the 256 MB last-level
// cache can hold (coefficients plus about six vectors).
// lcs_set_tiling overrides each choice.
struct Tuning {
    int march_rows, nontemporal;
};
MarchGeom march_geom(const Tuning &t, int64_t upr, int rows) {
    int64_t h = march_strips(upr) * (int64_t)rows / 2048;
    h = std::max<int64_t>(1, std::min<int64_t>(32, h));
    if (t.march_rows > 0) h = t.march_rows;
    return {(int)h};
}
// Walk mode of the stencil operators (see MarchGeom): row marching with
// non-temporal streams once the FP64 pass (coefficients plus about six
// vectors) exceeds the 256 MB last-level cache, else the flat walk, whose
// repeated row reads are cache hits there.
int walk_mode(const Tuning &t, const lcs_matrix *A, int n_arr) {
    const double bytes = (double)A->nx * A->ny * A->nz * (double)(n_arr + 6) * 8.0;
    int m = bytes > 256.0 * 1024 * 1024 ? 2 : 0;
    if (t.march_rows < 0) m = 0;
    else if (t.march_rows > 0) m = 2;
    if (m > 0 && t.nontemporal == 0) m = 1;
    return m;
}
template <typename real, int V, int W>
U5<real, V, W> uop5(const Tuning &t, const lcs_matrix *A, const real *c) {
    const int64_t n = (int64_t)A->nx * A->ny;
    return {c, c + n, c + 2 * n, A->nx, A->ny, n, march_geom(t, A->nx / V, A->ny)};
}
template <typename real, int V, int W>
U9<real, V, W> uop9(const Tuning &t, const lcs_matrix *A, const real *c) {
    const int64_t n = (int64_t)A->nx * A->ny;
    return {c, c + n, c + 2 * n, c + 3 * n, c + 4 * n, A->nx, A->ny, n, march_geom(t, A->nx / V, A->ny)};
}
template <typename real, int V, int W>
U7<real, V, W> uop7(const Tuning &t, const lcs_matrix *A, const real *c) {
    const int64_t n = (int64_t)A->nx * A->ny * A->nz;
    return {c, c + n, c + 2 * n, c + 3 * n, A->nx, A->ny, A->nz, n,
            march_geom(t, (int64_t)A->nx * A->ny / V, A->nz)};
}

template <int W>
struct Width {
    static constexpr int value = W;
};

bool aligned16(const void *p) { return p == nullptr || ((uintptr_t)p & 15u) == 0; }

// Calls f(scalar_op64, unit_op64, unit_op32, Width<W>) for A's kind.
template <class F>
lcs_status with_ops(const lcs_ctx *c, const lcs_matrix *A, const float *coef32, bool vec_ok, F &&f) {
    const bool v = vec_ok && A->nx % 4 == 0 && aligned16(A->coef) && aligned16(coef32);
    const Tuning t{c->march_rows, c->nontemporal};
    if (A->kind == LCS_CSR) {   // the ELL copy made by prepare_matrix
        const auto &E = c->ell;
        const float *d32 = coef32 ? coef32 + (int64_t)E.width * E.n : nullptr;
        // stream the copy once an FP64 pass (indices, values and about six
        // vectors) exceeds the 256 MB last-level cache
        const bool stream = (double)E.n * (E.width * 12.0 + 48.0) > 256.0 * 1024 * 1024;
        auto go = [&](auto wtag) -> lcs_status {
            constexpr int W = decltype(wtag)::value;
            const double *dg = E.val + (int64_t)W * E.n;
            const EllRows<double, W> rows{E.col, E.val, dg, E.clr, E.n};
            if (stream)
                return f(rows, UEllStream<double, W>{{E.col, E.val, dg, E.clr, E.n}},
                         UEllStream<float, W>{{E.col, coef32, d32, E.clr, E.n}}, wtag);
            return f(rows, UEll<double, W>{E.col, E.val, dg, E.clr, E.n},
                     UEll<float, W>{E.col, coef32, d32, E.clr, E.n}, wtag);
        };
        switch (E.width) {
        case 5: return go(Width<5>());
        case 7: return go(Width<7>());
        case 9: return go(Width<9>());
        case 16: return go(Width<16>());
        default: return go(Width<64>());
        }
    }
    switch (A->kind) {
    case LCS_STENCIL5_2D: {
        const auto s5 = sop5<double>(A, A->coef);
        if (!v) return f(s5, uop5<double, 1, 0>(t, A, A->coef), uop5<float, 1, 0>(t, A, coef32), Width<5>());
        switch (walk_mode(t, A, 3)) {
        case 0: return f(s5, uop5<double, 2, 0>(t, A, A->coef), uop5<float, 4, 0>(t, A, coef32), Width<5>());
        case 1: return f(s5, uop5<double, 2, 1>(t, A, A->coef), uop5<float, 4, 1>(t, A, coef32), Width<5>());
        default: return f(s5, uop5<double, 2, 2>(t, A, A->coef), uop5<float, 4, 2>(t, A, coef32), Width<5>());
        }
    }
    case LCS_STENCIL9_2D: {
        const auto s9 = sop9<double>(A, A->coef);
        if (!v) return f(s9, uop9<double, 1, 0>(t, A, A->coef), uop9<float, 1, 0>(t, A, coef32), Width<9>());
        switch (walk_mode(t, A, 5)) {
        case 0: return f(s9, uop9<double, 2, 0>(t, A, A->coef), uop9<float, 4, 0>(t, A, coef32), Width<9>());
        case 1: return f(s9, uop9<double, 2, 1>(t, A, A->coef), uop9<float, 4, 1>(t, A, coef32), Width<9>());
        default: return f(s9, uop9<double, 2, 2>(t, A, A->coef), uop9<float, 4, 2>(t, A, coef32), Width<9>());
        }
    }
    case LCS_STENCIL9N_2D:
        // full storage, flat walk, one row per unit (GMRES vectors)
        return f(sop9n<double>(A, A->coef), uop9n<double>(A, A->coef), uop9n<float>(A, coef32),
                 Width<9>());
    default: {
        const auto s7 = sop7<double>(A, A->coef);
        if (!v) return f(s7, uop7<double, 1, 0>(t, A, A->coef), uop7<float, 1, 0>(t, A, coef32), Width<7>());
        switch (walk_mode(t, A, 4)) {
        case 0: return f(s7, uop7<double, 2, 0>(t, A, A->coef), uop7<float, 4, 0>(t, A, coef32), Width<7>());
        case 1: return f(s7, uop7<double, 2, 1>(t, A, A->coef), uop7<float, 4, 1>(t, A, coef32), Width<7>());
        default: return f(s7, uop7<double, 2, 2>(t, A, A->coef), uop7<float, 4, 2>(t, A, coef32), Width<7>());
        }
    }
    }
}

// General sparse input: check the structure (one synchronisation, before
// any kernel reads through the column indices), then copy A into
// column-major ELL of width 5, 7, 9, 16 or 64 in the context.  Stencil kinds:
// nothing.
lcs_status prepare_matrix(lcs_ctx *c, const lcs_matrix *A, hipStream_t s) {
    if (A->kind != LCS_CSR) return LCS_OK;
    const int64_t n = A->nx;
    auto &E = c->ell;
    if (A->csr_reuse && E.valid && E.n == n && E.rp == A->row_ptr && E.col_in == A->col &&
        E.val_in == A->val && E.clr_in == A->colour && E.nnz == A->nnz && E.ncol == A->n_colours)
        return LCS_OK;
    E.valid = false;
    int32_t *flags;
    LCS_TRY(get_buf(c, B_AFLAGS, 2, &flags));
    hipLaunchKernelGGL(k_fill<int32_t>, dim3(1), dim3(kBlock), 0, s, flags, 0, (int64_t)2);
    hipLaunchKernelGGL(k_csr_check, dim3(std::min(flat_grid(n), kMaxGrid)), dim3(kBlock), 0, s,
                       A->row_ptr, A->col, A->val, n, A->nnz, A->colour, A->n_colours,
                       A->csr_nonsym ? 1 : 0, flags);
    LAUNCH_CHECK();
    int32_t h[2] = {0, 0};
    HIP_TRY(hipMemcpyAsync(h, flags, sizeof(h), hipMemcpyDeviceToHost, s));
    LCS_TRY(wait_for(c, s));
    if (h[0]) {
        std::string m = "CSR matrix:";
        if (h[0] & kCsrBadPtr) m += " row_ptr not non-decreasing in [0, nnz];";
        if (h[0] & kCsrEnds) m += " row_ptr[0] != 0 or row_ptr[N] != nnz;";
        if (h[0] & kCsrEmpty) m += " empty row;";
        if (h[0] & kCsrLong) m += " row longer than 64 entries;";
        if (h[0] & kCsrCol) m += " column out of range;";
        if (h[0] & kCsrOrder) m += " columns not strictly ascending;";
        if (h[0] & kCsrNoDiag) m += " diagonal entry missing;";
        if (h[0] & kCsrColour) m += " colouring invalid (colour >= n_colours or two coupled rows share one);";
        if (h[0] & kCsrBadDiag)
            m += A->csr_nonsym ? " zero diagonal entry;" : " diagonal entry <= 0 (not SPD);";
        if (h[0] & kCsrNonFinite) m += " NaN or infinite value;";
        // a well-formed matrix whose only fault is a non-finite value
        return fail(h[0] == kCsrNonFinite ? LCS_ENONFINITE : LCS_EINVAL, m);
    }
    // the widths of the stencil kinds, whose ELL operators the local
    // systems already use, then 16, then 64 for rows of up to 64 entries
    // (a row's entries stay in registers: at 64 the kernels spill, a
    // fallback for rare long rows rather than a tuned path)
    const int W = h[1] <= 5 ? 5 : h[1] <= 7 ? 7 : h[1] <= 9 ? 9 : h[1] <= 16 ? 16 : 64;
    LCS_TRY(get_buf(c, B_ACOL, (size_t)W * n, &c->ell.col));
    LCS_TRY(get_buf(c, B_AVAL, (size_t)(W + 1) * n, &c->ell.val));
    LCS_TRY(get_buf(c, B_ACLR, (size_t)n, &c->ell.clr));
    auto conv = [&](auto kernel) {
        hipLaunchKernelGGL(kernel, dim3(flat_grid(n)), dim3(kBlock), 0, s, A->row_ptr, A->col,
                           A->val, n, A->colour, c->ell.col, c->ell.val, c->ell.clr);
    };
    switch (W) {
    case 5: conv(k_csr_to_ell<5>); break;
    case 7: conv(k_csr_to_ell<7>); break;
    case 9: conv(k_csr_to_ell<9>); break;
    case 16: conv(k_csr_to_ell<16>); break;
    default: conv(k_csr_to_ell<64>); break;
    }
    LAUNCH_CHECK();
    E.width = W;
    E.n = n;
    E.rp = A->row_ptr;
    E.col_in = A->col;
    E.val_in = A->val;
    E.clr_in = A->colour;
    E.nnz = A->nnz;
    E.ncol = A->n_colours;
    E.valid = true;
    return LCS_OK;
}

lcs_status ensure_coef32(lcs_ctx *c, const lcs_matrix *A, bool need, const float **out,
                         hipStream_t s) {
    *out = nullptr;
    if (!need) return LCS_OK;
    if (A->kind == LCS_CSR) {   // FP32 copy of the ELL values and the diagonal
        const int64_t m = (int64_t)(c->ell.width + 1) * c->ell.n;
        float *p;
        LCS_TRY(get_buf(c, B_COEF32, (size_t)m, &p));
        hipLaunchKernelGGL(k_cast, dim3(flat_grid(m)), dim3(kBlock), 0, s, (const double *)c->ell.val,
                           p, m);
        LAUNCH_CHECK();
        *out = p;
        return LCS_OK;
    }
    if (A->coef32) {
        *out = A->coef32;
        return LCS_OK;
    }
    const int64_t n = (int64_t)A->nx * A->ny * A->nz * n_arrays(A->kind);
    float *p;
    LCS_TRY(get_buf(c, B_COEF32, (size_t)n, &p));
    hipLaunchKernelGGL(k_cast, dim3(flat_grid(n)), dim3(kBlock), 0, s, A->coef, p, n);
    LAUNCH_CHECK();
    *out = p;
    return LCS_OK;
}

lcs_status launch_norm(lcs_ctx *c, const double *v, int64_t n, double *out, hipStream_t s) {
    const Launch L = dims_wide(n, 4096);   // one partial per block
    hipLaunchKernelGGL(k_norm2, dim3(L.grid), dim3(kBlock), 0, s, v, n, L.chunk, slot(c, kPtNorm));
    hipLaunchKernelGGL(k_fin_norm, dim3(1), dim3(kBlock), 0, s, (const double *)slot(c, kPtNorm),
                       L.grid, out);
    LAUNCH_CHECK();
    return LCS_OK;
}

// ---------------------------------------------------------------------------
// PCG driver
// ---------------------------------------------------------------------------
template <typename real>
struct PcgBufs {
    real *r, *z, *p0, *p1, *q;
    real *w0, *w1, *s0, *s1;   // single-synchronisation PCG
};

struct PcgResult {
    int its = 0;
    int status = kStOk;
};

// z = M^-1 r for the symmetric red-black (or four-colour) Gauss-Seidel
// preconditioner from z = 0: colours 0..nc-1, then nc-2..0 (the backward
// pass's first colour would repeat the forward pass's last one exactly).
// Whether op is the restricted system of the current local solve with its
// rows blocked by colour (see local_phase).
template <class Op>
bool colour_blocked(const lcs_ctx *c, const Op &A, int ncol) {
    if constexpr (is_ell<Op>) {
        return c->cblk.n == ncol && ncol >= 2 && c->cblk.start[ncol] == A.n;
    } else {
        return false;
    }
}

template <class Op, int kPc>
lcs_status launch_precond(lcs_ctx *c, const Op &A, const PcgBufs<typename Op::real> &B, int grid,
                          int ncol, hipStream_t s) {
    using real = typename Op::real;
    if (kPc != LCS_PC_RBSGS) return LCS_OK;
    real *part = slot_as<real>(c, kPtSgs);
    const Scalars *sc = c->dsc;
    if constexpr (is_ell<Op>) {
        if (colour_blocked(c, A, ncol)) {
            // a restricted system with its rows blocked by colour: each half
            // sweep reads its colour's rows only, and each colour's last update
            // (colour ncol-1 forward, the others backward) writes the r.z
            // partials of its rows into a set of its own
            const auto &cb = c->cblk;
            auto half = [&](int col, int set) {
                if (set >= 0)
                    hipLaunchKernelGGL((k_gs_half_blk<Op, true>), dim3(grid), dim3(kBlock), 0, s, A,
                                       (const real *)B.r, B.z, cb.start[col], cb.start[col + 1], sc,
                                       part + (size_t)set * grid);
                else
                    hipLaunchKernelGGL((k_gs_half_blk<Op, false>), dim3(grid), dim3(kBlock), 0, s, A,
                                       (const real *)B.r, B.z, cb.start[col], cb.start[col + 1], sc,
                                       part);
            };
            for (int col = 1; col < ncol; ++col) half(col, col == ncol - 1 ? 0 : -1);
            for (int col = ncol - 2; col >= 0; --col) half(col, ncol - 1 - col);
            LAUNCH_CHECK();
            return LCS_OK;
        }
    }
    // colour 0 of the forward sweep is done by the kernel that formed r.
    // One colour (a diagonal matrix with a one-class colouring): the backward
    // pass is colour 0 again, which reproduces z bit for bit and writes the
    // r.z partials.
    if (ncol == 1) {
        hipLaunchKernelGGL((k_gs_half<Op, true>), dim3(grid), dim3(kBlock), 0, s, A,
                           (const real *)B.r, B.z, 0, sc, part);
        LAUNCH_CHECK();
        return LCS_OK;
    }
    for (int col = 1; col < ncol; ++col)
        hipLaunchKernelGGL((k_gs_half<Op, false>), dim3(grid), dim3(kBlock), 0, s, A,
                           (const real *)B.r, B.z, col, sc, part);
    for (int col = ncol - 2; col >= 0; --col) {
        if (col == 0)
            hipLaunchKernelGGL((k_gs_half<Op, true>), dim3(grid), dim3(kBlock), 0, s, A,
                               (const real *)B.r, B.z, col, sc, part);
        else
            hipLaunchKernelGGL((k_gs_half<Op, false>), dim3(grid), dim3(kBlock), 0, s, A,
                               (const real *)B.r, B.z, col, sc, part);
    }
    LAUNCH_CHECK();
    return LCS_OK;
}

// PCG on op x = rhs.  Convergence lives on the device: iteration j is
// k_pcg_ap(j) + k_pcg_update(j), and the stopping test of the iterate after
// update(j-1) runs at the start of ap(j).  The host enqueues check_every
// iterations at a time and polls the flag of the previous chunk while the
// next one runs, so the GPU never waits for the host; launches after
// convergence exit at their first instruction.
// Launch one kernel; when kernel timing is on for its class, through
// hipExtLaunchKernelGGL with a start / stop event pair that the dispatch
// itself records (so the interval is the kernel's execution, not the host's
// launch latency).
template <class K, class... Args>
lcs_status launch_maybe_timed(lcs_ctx *c, bool timed, K kernel, int grid, hipStream_t s,
                              Args... args) {
    if (!timed) {
        hipLaunchKernelGGL(kernel, dim3(grid), dim3(kBlock), 0, s, args...);
        LAUNCH_CHECK();
        return LCS_OK;
    }
    while (c->prof_ev.size() < c->prof_used + 2) {
        hipEvent_t e;
        HIP_TRY(hipEventCreate(&e));
        c->prof_ev.push_back(e);
    }
    hipEvent_t e0 = c->prof_ev[c->prof_used++];
    hipEvent_t e1 = c->prof_ev[c->prof_used++];
    hipExtLaunchKernelGGL(kernel, dim3(grid), dim3(kBlock), 0, s, e0, e1, 0, args...);
    LAUNCH_CHECK();
    return LCS_OK;
}

// After the stream is idle: fold the recorded event pairs into the totals.
lcs_status flush_prof(lcs_ctx *c) {
    for (size_t k = 0; k + 1 < c->prof_used; k += 2) {
        float ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms, c->prof_ev[k], c->prof_ev[k + 1]));
        c->prof_ms += ms;
        c->prof_launches += 1;
    }
    c->prof_used = 0;
    return LCS_OK;
}

// A caller's work that follows a PCG solve on the stream and ends with a
// copy of the scalars to hsc and a record_done (see run_chunks).
using Tail = std::function<lcs_status()>;

// Enqueue PCG iterations in chunks between host checks, with up to two
// chunks in flight: the host waits for the older chunk while the newer one
// runs, so the GPU does not wait for the host.  launch(j) enqueues iteration
// j; launch(max_iter) is the final stopping test.  After each chunk the PCG
// state (stop flag, recursive residual, tolerance) is copied to pinned host
// memory.  The first chunk is sized from the previous solve of the same
// kind and step; later chunks from the residual's decay so far, so that few
// launches run (and exit at once) after convergence.
// tail (optional): enqueued right behind the chunk after which the solve is
// expected to have stopped; its kernels must do nothing while the stop flag
// is unset.  No chunk is enqueued behind it: the host waits for the tail,
// and if the solve had not stopped, enqueues more chunks and the tail again.
// *tailed: the solve ended with a tail that ran after the stop (hsc holds
// its copy); otherwise the caller does that work itself.
template <class F>
lcs_status run_chunks(lcs_ctx *c, hipStream_t s, int max_iter, int check_every, int prev_its,
                      F &&launch, const Tail *tail = nullptr, bool *tailed = nullptr) {
    int next_j = 0, nin = 0;
    int inflight[2] = {0, 1}, launched_at[2] = {0, 0};
    bool tail_in = false;
    if (tailed) *tailed = false;
    bool known = false;
    int known_it = 0;
    double rho = 0.0, rho0 = 0.0, tol = 0.0;
    // launches the solve is expected to need in total (two over the estimate:
    // a launch that exits at once costs less than a host round trip)
    auto estimate = [&]() -> int {
        if (!known) return prev_its > 0 ? prev_its + 2 : next_j + check_every;
        const double q = std::pow(rho / rho0, 1.0 / std::max(known_it, 1));
        if (!(q > 0.0) || !(q < 1.0) || !(tol > 0.0) || !(rho > tol))
            return known_it + 1 + check_every;
        const double rest = std::ceil(std::log(tol / rho) / std::log(q));
        return known_it + 2 + (int)std::min(rest, 4.0 * check_every);
    };
    auto enqueue = [&](int len) -> lcs_status {
        const int sl = nin == 0 ? 0 : inflight[0] ^ 1;
        for (int k = 0; k < len && next_j < max_iter; ++k) LCS_TRY(launch(next_j++));
        if (next_j >= max_iter) LCS_TRY(launch(next_j));   // final stopping test
        launched_at[sl] = next_j;
        HIP_TRY(hipMemcpyAsync(&c->hpcg[sl], &c->dsc->pcg, sizeof(PcgState),
                               hipMemcpyDeviceToHost, s));
        HIP_TRY(hipEventRecord(c->chk[sl], s));
        inflight[nin++] = sl;
        return LCS_OK;
    };
    // the tail, once the chunks enqueued so far are expected to end the
    // solve (always after the final stopping test)
    auto maybe_tail = [&]() -> lcs_status {
        if (!tail || tail_in || (next_j < max_iter && next_j < estimate())) return LCS_OK;
        LCS_TRY((*tail)());
        tail_in = true;
        return LCS_OK;
    };
    LCS_TRY(enqueue(std::max(check_every, prev_its - check_every / 2)));
    LCS_TRY(maybe_tail());
    for (;;) {
        if (!tail_in && nin < 2 && next_j < max_iter) {
            const int len = std::min(check_every, estimate() - next_j);
            if (len > 0) {
                LCS_TRY(enqueue(len));
                LCS_TRY(maybe_tail());
            }
        }
        if (nin == 0) {
            // only the tail is in flight, behind a chunk that ended unstopped
            // (the tail left everything as it was): go on after it
            if (!tail_in) return fail(LCS_EHIP, "PCG driver: nothing in flight");
            LCS_TRY(wait_recorded(c, s));
            tail_in = false;
            LCS_TRY(enqueue(std::max(1, std::min(check_every, estimate() - next_j))));
            LCS_TRY(maybe_tail());
            continue;
        }
        const int sl = inflight[0];
        LCS_TRY(spin_event(c->chk[sl]));
        inflight[0] = inflight[1];
        --nin;
        const PcgState &h = c->hpcg[sl];
        if (h.done) {
            if (tail_in) {   // the tail runs after the stop
                LCS_TRY(wait_recorded(c, s));
                *tailed = true;
            }
            break;
        }
        // the last launch of the chunk tested the residual of iterate
        // launched_at - 1
        known = true;
        known_it = launched_at[sl] - 1;
        rho = std::sqrt(h.rr);
        rho0 = std::sqrt(h.rr0);
        tol = h.tol;
        if (nin == 0 && !tail_in) {
            if (next_j >= max_iter) break;   // not reached: the final test sets the flag
            LCS_TRY(enqueue(std::max(1, std::min(check_every, estimate() - next_j))));
            LCS_TRY(maybe_tail());
        }
    }
    return LCS_OK;
}

int &last_its_of(lcs_ctx *c, int scope) { return c->last_its[scope][std::min(c->cur_outer, 3)]; }

// Single-synchronisation PCG (Jacobi / none): k_cg_init1, k_cg_init2, then
// one k_cg_iter per iteration; the stopping test of x_j runs at the start of
// iteration j.  Buffers: r, w, s double-buffered by iteration parity.
// prepared: the caller already zeroed x, put rhs into B.r and reset the PCG
// state (k_refine_start), so the solve starts at k_cg_init2.  save: keep
// the outcome in saved_it / saved_status[scope] here (else the caller's
// next kernel does, as k_axpy_scaled does).
template <class Op, int kPc>
lcs_status run_cg1(lcs_ctx *c, const Op &A, const typename Op::real *rhs, typename Op::real *x,
                   bool x_zero, const double *tol_base, double tol_factor, int max_iter,
                   int check_every, const PcgBufs<typename Op::real> &B, hipStream_t s,
                   PcgResult *res, int scope, bool sync_end, bool save, bool prepared,
                   const Tail *tail, bool *tailed) {
    using real = typename Op::real;
    const int64_t n = A.units() * Op::V;
    const int grid = grid_for(A, kRedGrid);
    real *part[2] = {slot_as<real>(c, kPtAp), slot_as<real>(c, kPtUpd)};
    real *r[2] = {B.r, B.z}, *w[2] = {B.w0, B.w1}, *sv[2] = {B.s0, B.s1};
    if (max_iter < 0) max_iter = 0;
    if (!prepared) {
        if (x_zero) {
            hipLaunchKernelGGL(k_fill<real>, dim3(flat_grid(n)), dim3(kBlock), 0, s, x, real(0), n);
            LAUNCH_CHECK();
        }
        hipLaunchKernelGGL((k_cg_init1<Op, kPc>), dim3(grid), dim3(kBlock), 0, s, A, rhs,
                           (const real *)x, r[0], x_zero ? 1 : 0, c->dsc);
    }
    hipLaunchKernelGGL((k_cg_init2<Op, kPc>), dim3(grid), dim3(kBlock), 0, s, A,
                       (const real *)r[0], w[0], part[0]);
    LAUNCH_CHECK();
    if (check_every < 1) check_every = 1;
    const bool timed = c->prof_what == (scope == 1 ? LCS_TIME_LOCAL_AP : LCS_TIME_GLOBAL_AP);
    auto launch_iter = [&](int j) -> lcs_status {
        const int a = j & 1, b = a ^ 1;
        return launch_maybe_timed(c, timed, k_cg_iter<Op, kPc>, grid, s, A, x, B.p0,
                                  (const real *)sv[b], sv[a], (const real *)r[a], r[b],
                                  (const real *)w[a], w[b], j, max_iter, tol_base, tol_factor,
                                  c->dsc, (const real *)part[a], part[b]);
    };
    LCS_TRY(run_chunks(c, s, max_iter, check_every, last_its_of(c, scope), launch_iter, tail,
                       tailed));
    if (save) {
        hipLaunchKernelGGL(k_save_pcg, dim3(1), dim3(1), 0, s, c->dsc, scope);
        LAUNCH_CHECK();
    }
    if (!sync_end) {
        res->its = -1;
        res->status = kStOk;
        return LCS_OK;
    }
    LCS_TRY(read_scalars(c, s));
    res->its = c->hsc->saved_it[scope];
    res->status = c->hsc->saved_status[scope];
    last_its_of(c, scope) = res->its;
    return LCS_OK;
}

template <class Op, int kPc>
lcs_status run_pcg_t(lcs_ctx *c, const Op &A, int ncol, const typename Op::real *rhs,
                     typename Op::real *x, bool x_zero, const double *tol_base, double tol_factor,
                     int max_iter, int check_every, const PcgBufs<typename Op::real> &B,
                     hipStream_t s, PcgResult *res, int scope, bool sync_end, bool save,
                     const Tail *tail, bool *tailed) {
    using real = typename Op::real;
    const int64_t n = A.units() * Op::V;
    const int grid = grid_for(A, kRedGrid);
    real *pupd = slot_as<real>(c, kPtUpd), *pap = slot_as<real>(c, kPtAp);
    real *psgs = slot_as<real>(c, kPtSgs);
    // the r.z partials of the preconditioner: one set per colour when the
    // rows are blocked by colour, else one
    const int gsgs = colour_blocked(c, A, ncol) ? ncol * grid : grid;
    if (max_iter < 0) max_iter = 0;
    if (x_zero) {
        hipLaunchKernelGGL(k_fill<real>, dim3(flat_grid(n)), dim3(kBlock), 0, s, x, real(0), n);
        LAUNCH_CHECK();
    }
    hipLaunchKernelGGL((k_pcg_init<Op, kPc>), dim3(grid), dim3(kBlock), 0, s, A, rhs,
                       (const real *)x, B.r, B.z, x_zero ? 1 : 0, c->dsc, pupd);
    LAUNCH_CHECK();
    LCS_TRY((launch_precond<Op, kPc>(c, A, B, grid, ncol, s)));
    if (check_every < 1) check_every = 1;
    int flip = 0;
    const bool time_ap = c->prof_what == (scope == 1 ? LCS_TIME_LOCAL_AP : LCS_TIME_GLOBAL_AP);
    const bool time_up = c->prof_what == (scope == 1 ? LCS_TIME_LOCAL_UPDATE : LCS_TIME_GLOBAL_UPDATE);
    auto launch_ap = [&](int j) -> lcs_status {
        real *pold = flip ? B.p1 : B.p0;
        real *pnew = flip ? B.p0 : B.p1;
        return launch_maybe_timed(c, time_ap, k_pcg_ap<Op, kPc>, grid, s, A, (const real *)B.z,
                                  (const real *)pold, pnew, B.q, j, max_iter, tol_base, tol_factor,
                                  c->dsc, (const real *)pupd, (const real *)psgs, gsgs, pap);
    };
    // iteration j: q = A p (with the stopping test), the update, the
    // preconditioner; j == max_iter: the final stopping test alone
    auto launch_iter = [&](int j) -> lcs_status {
        LCS_TRY(launch_ap(j));
        if (j >= max_iter) return LCS_OK;
        real *pnew = flip ? B.p0 : B.p1;
        LCS_TRY(launch_maybe_timed(c, time_up, k_pcg_update<Op, kPc>, grid, s, A, x,
                                   (const real *)pnew, (const real *)B.q, B.r, B.z, j, c->dsc,
                                   (const real *)pap, pupd));
        LCS_TRY((launch_precond<Op, kPc>(c, A, B, grid, ncol, s)));
        flip ^= 1;
        return LCS_OK;
    };
    LCS_TRY(run_chunks(c, s, max_iter, check_every, last_its_of(c, scope), launch_iter, tail,
                       tailed));
    if (save) {
        hipLaunchKernelGGL(k_save_pcg, dim3(1), dim3(1), 0, s, c->dsc, scope);
        LAUNCH_CHECK();
    }
    if (!sync_end) {   // the caller reads saved_it / saved_status later
        res->its = -1;
        res->status = kStOk;
        return LCS_OK;
    }
    LCS_TRY(read_scalars(c, s));
    res->its = c->hsc->saved_it[scope];
    res->status = c->hsc->saved_status[scope];
    last_its_of(c, scope) = res->its;
    return LCS_OK;
}

template <class Op>
lcs_status run_pcg(lcs_ctx *c, const Op &A, int ncol, int pc, const typename Op::real *rhs,
                   typename Op::real *x, bool x_zero, const double *tol_base, double tol_factor,
                   int max_iter, int check_every, const PcgBufs<typename Op::real> &B,
                   hipStream_t s, PcgResult *res, int scope, bool sync_end, bool save = true,
                   bool prepared = false, const Tail *tail = nullptr, bool *tailed = nullptr) {
    switch (pc) {
    case LCS_PC_NONE:
        return run_cg1<Op, 0>(c, A, rhs, x, x_zero, tol_base, tol_factor, max_iter, check_every, B,
                              s, res, scope, sync_end, save, prepared, tail, tailed);
    case LCS_PC_JACOBI:
        return run_cg1<Op, 1>(c, A, rhs, x, x_zero, tol_base, tol_factor, max_iter, check_every, B,
                              s, res, scope, sync_end, save, prepared, tail, tailed);
    default:   // the caller never prepares this one (k_pcg_init also starts z)
        return run_pcg_t<Op, 2>(c, A, ncol, rhs, x, x_zero, tol_base, tol_factor, max_iter,
                                check_every, B, s, res, scope, sync_end, save, tail, tailed);
    }
}

lcs_status status_of(int st) {
    switch (st) {
    case kStOk: return LCS_OK;
    case kStNoConv: return fail(LCS_ENOCONV, "iteration limit reached before the criterion");
    case kStBreakdown: return fail(LCS_EBREAKDOWN, "p^T A p <= 0: operator not SPD");
    default: return fail(LCS_ENONFINITE, "non-finite value in the iteration");
    }
}

template <class Op>
lcs_status launch_resnorm(lcs_ctx *c, const Op &A, const double *rhs, const double *x, double *r,
                          const double *tol_base, double tol_factor, hipStream_t s) {
    const int grid = grid_for(A, kRedGrid);
    hipLaunchKernelGGL((k_resnorm<Op>), dim3(grid), dim3(kBlock), 0, s, A, rhs, x, r,
                       slot(c, kPtRes));
    hipLaunchKernelGGL(k_fin_res, dim3(1), dim3(kBlock), 0, s, (const double *)slot(c, kPtRes),
                       grid, tol_base, tol_factor, c->dsc);
    LAUNCH_CHECK();
    return LCS_OK;
}

struct SolveOut {
    int its = 0;
    int n_outer = 0;
    double rr = 0.0;  // ||rhs - op x||^2 at exit (FP64)
};

// Solve op x = rhs to ||rhs - op x|| <= tol_factor * *tol_base.
// FP64: PCG, then a true-residual check with up to max_outer restarts.
// Mixed: FP64 residual -> scaled FP32 PCG correction to inner_tol -> FP64
// update, repeated until the FP64 criterion holds.
// scope 0 (global): after PCG the true residual is checked, with restarts.
// scope 1 (local, FP64): one PCG run with no host round trip; its outcome is
// left in saved_it[1] / saved_status[1] for the caller's next read (the
// criterion that matters is the global one checked right after).
template <class Op64, class Op32>
lcs_status solve_system_sym(lcs_ctx *c, const Op64 &A, const Op32 &A32, int ncol, const double *rhs,
                        double *x, bool x_zero, const double *tol_base, double tol_factor,
                        const lcs_options *o, hipStream_t s, SolveOut *out, int scope) {
    const int64_t n = A.units() * Op64::V;
    *out = SolveOut();
    if (n == 0) return LCS_OK;
    const int check = o->check_every > 0 ? o->check_every : 8;
    if (o->precision == LCS_PREC_FP64) {
        PcgBufs<double> B;
        LCS_TRY(get_buf(c, B_R, n, &B.r));
        LCS_TRY(get_buf(c, B_Z, n, &B.z));
        LCS_TRY(get_buf(c, B_P0, n, &B.p0));
        LCS_TRY(get_buf(c, B_P1, n, &B.p1));
        LCS_TRY(get_buf(c, B_Q, n, &B.q));
        LCS_TRY(get_buf(c, B_W0, n, &B.w0));
        LCS_TRY(get_buf(c, B_W1, n, &B.w1));
        LCS_TRY(get_buf(c, B_S0, n, &B.s0));
        LCS_TRY(get_buf(c, B_S1, n, &B.s1));
        if (scope == 1) {
            PcgResult pr;
            c->cur_outer = 0;
            LCS_TRY(run_pcg(c, A, ncol, o->precond, rhs, x, x_zero, tol_base, tol_factor,
                            o->max_iter, check, B, s, &pr, scope, false));
            out->its = -1;
            return LCS_OK;
        }
        bool zero = x_zero;
        for (int attempt = 0;; ++attempt) {
            PcgResult pr;
            c->cur_outer = attempt;
            LCS_TRY(run_pcg(c, A, ncol, o->precond, rhs, x, zero, tol_base, tol_factor,
                            o->max_iter - out->its, check, B, s, &pr, scope, true));
            zero = false;
            out->its += pr.its;
            LCS_TRY(launch_resnorm(c, A, rhs, x, (double *)nullptr, tol_base, tol_factor, s));
            LCS_TRY(read_scalars(c, s));
            out->rr = c->hsc->res.rr;
            if (pr.status != kStOk) return status_of(pr.status);
            if (c->hsc->res.status != kStOk) return status_of(c->hsc->res.status);
            if (c->hsc->res.done) return LCS_OK;
            if (attempt >= o->max_outer || out->its >= o->max_iter) return status_of(kStNoConv);
            out->n_outer += 1;
        }
    }
    double *r64;
    float *r32, *d32;
    PcgBufs<float> B;
    LCS_TRY(get_buf(c, B_RES, n, &r64));
    LCS_TRY(get_buf(c, B_R32, n, &r32));
    LCS_TRY(get_buf(c, B_D32, n, &d32));
    LCS_TRY(get_buf(c, B_RI32, n, &B.r));
    LCS_TRY(get_buf(c, B_Z32, n, &B.z));
    LCS_TRY(get_buf(c, B_P32A, n, &B.p0));
    LCS_TRY(get_buf(c, B_P32B, n, &B.p1));
    LCS_TRY(get_buf(c, B_Q32, n, &B.q));
    LCS_TRY(get_buf(c, B_W32A, n, &B.w0));
    LCS_TRY(get_buf(c, B_W32B, n, &B.w1));
    LCS_TRY(get_buf(c, B_S32A, n, &B.s0));
    LCS_TRY(get_buf(c, B_S32B, n, &B.s1));
    const double inner = o->inner_tol > 0 ? o->inner_tol : 1e-5;
    const int outer_cap = o->max_outer > 0 ? o->max_outer : 10;
    if (x_zero) {
        hipLaunchKernelGGL(k_fill<double>, dim3(flat_grid(n)), dim3(kBlock), 0, s, x, 0.0, n);
        LAUNCH_CHECK();
    }
    // The outcome of each inner PCG (iterations, status) stays on the device
    // until the host reads the next FP64 residual: one host round trip per
    // refinement step.  The first step is enqueued before its residual is
    // read: k_refine_start (or k_cast_scale) turns it into a no-op (zero
    // right-hand side, the inner solve stops at its first test, x unchanged)
    // when that residual already meets the criterion or is non-finite, and
    // the next read then ends the solve exactly as a read before the step
    // would have.
    int pending = -1;   // refinement step whose inner outcome is not yet read
    auto settle = [&]() -> lcs_status {
        if (pending < 0) return LCS_OK;
        const int it = c->hsc->saved_it[scope];
        const int ps = c->hsc->saved_status[scope];
        const int step = pending;
        pending = -1;
        if (ps == kStBreakdown || ps == kStNonFinite) {
            out->its += it;
            return status_of(ps);
        }
        if (it == 0) {   // the no-op first step (a non-zero residual takes >= 1 iteration)
            out->n_outer -= 1;
            return LCS_OK;
        }
        out->its += it;
        c->last_its[scope][std::min(step, 3)] = it;
        return LCS_OK;
    };
    // A step's update, the next step's FP64 residual and the read of both
    // form the step's tail: the PCG driver enqueues it behind the iterations
    // it expects the inner solve to need (the update waits on the inner
    // solve's stop flag), so one host round trip serves the end of the inner
    // solve and the criterion.
    bool have_res = false;   // the previous step's tail formed and read this step's residual
    const Tail tail = [&]() -> lcs_status {
        hipLaunchKernelGGL(k_axpy_scaled, dim3(flat_grid(n)), dim3(kBlock), 0, s, x,
                           (const float *)d32, n, c->dsc, scope);
        LAUNCH_CHECK();
        LCS_TRY(launch_resnorm(c, A, rhs, x, r64, tol_base, tol_factor, s));
        HIP_TRY(hipMemcpyAsync(c->hsc, c->dsc, sizeof(Scalars), hipMemcpyDeviceToHost, s));
        return record_done(c, s);
    };
    for (int outer = 0;; ++outer) {
        if (!have_res) LCS_TRY(launch_resnorm(c, A, rhs, x, r64, tol_base, tol_factor, s));
        const bool early = outer == 0 && o->max_iter > 0;
        if (!early) {
            if (!have_res) LCS_TRY(read_scalars(c, s));
            LCS_TRY(settle());
            out->rr = c->hsc->res.rr;
            if (c->hsc->res.status != kStOk) return status_of(c->hsc->res.status);
            if (c->hsc->res.done) return LCS_OK;
            if (outer >= outer_cap || out->its >= o->max_iter) return status_of(kStNoConv);
        }
        // the single-sync PCG starts from k_refine_start's r_0; the
        // Gauss-Seidel-preconditioned one from the scaled right-hand side
        const bool prep = o->precond != LCS_PC_RBSGS;
        if (prep)
            hipLaunchKernelGGL(k_refine_start, dim3(flat_grid(n)), dim3(kBlock), 0, s,
                               (const double *)r64,
                               o->precond == LCS_PC_JACOBI ? A32.diag_ptr() : (const float *)nullptr,
                               B.r, d32, n, c->dsc, early ? 1 : 0);
        else
            hipLaunchKernelGGL(k_cast_scale, dim3(flat_grid(n)), dim3(kBlock), 0, s,
                               (const double *)r64, r32, n, c->dsc, early ? 1 : 0);
        LAUNCH_CHECK();
        PcgResult pr;
        c->cur_outer = outer;
        bool tailed = false;
        LCS_TRY(run_pcg(c, A32, ncol, o->precond, (const float *)r32, d32, true,
                        (const double *)nullptr, inner, o->max_iter - out->its, check, B, s, &pr,
                        scope, false, false, prep, &tail, &tailed));
        if (!tailed) {
            hipLaunchKernelGGL(k_axpy_scaled, dim3(flat_grid(n)), dim3(kBlock), 0, s, x,
                               (const float *)d32, n, c->dsc, scope);
            LAUNCH_CHECK();
        }
        have_res = tailed;
        pending = outer;
        out->n_outer += 1;
    }
}


// Restarted GMRES(m) on a non-symmetric operator (see lcs_gmres.h): cycles
// of at most m Arnoldi steps, enqueued in chunks of check_every steps with a
// read of the done flag in between; after the residual estimate meets the
// tolerance the true residual is checked, and a failed check restarts (at
// most max_outer times), as for PCG.
template <class Op, int kPc>
lcs_status run_gmres_t(lcs_ctx *c, const Op &A, const double *rhs, double *x, bool x_zero,
                       const double *tol_base, double tol_factor, const lcs_options *o,
                       hipStream_t s, SolveOut *out) {
    const int64_t n = A.units();
    const int m = std::max(1, std::min(o->restart > 0 ? o->restart : 40, kMaxRestart));
    double *V, *W0, *W1, *ph0, *pn;
    GmState *st;
    LCS_TRY(get_buf(c, B_GMV, (size_t)(m + 1) * n, &V));
    LCS_TRY(get_buf(c, B_GMW0, n, &W0));
    LCS_TRY(get_buf(c, B_GMW1, n, &W1));
    LCS_TRY(get_buf(c, B_GMP0, (size_t)kGmPartVals * kGmGrid, &ph0));
    LCS_TRY(get_buf(c, B_GMPN, (size_t)kGmGrid, &pn));
    LCS_TRY(get_buf(c, B_GMS, 1, &st));
    const int g = band_grid(n, kGmGrid);
    const int check = o->check_every > 0 ? o->check_every : 8;
    if (x_zero) {
        hipLaunchKernelGGL(k_fill<double>, dim3(flat_grid(n)), dim3(kBlock), 0, s, x, 0.0, n);
        LAUNCH_CHECK();
    }
    bool from_zero = x_zero;
    int outer = 0;
    for (;;) {
        const int steps = (int)std::min<int64_t>(m, (int64_t)o->max_iter - out->its);
        hipLaunchKernelGGL((k_gm_init<Op>), dim3(g), dim3(kBlock), 0, s, A, rhs,
                           from_zero ? (const double *)nullptr : (const double *)x, W0, pn, st,
                           tol_base, tol_factor);
        hipLaunchKernelGGL(k_gm_fold_n, dim3(1), dim3(kBlock), 0, s, (const double *)pn, g, 0, st);
        LAUNCH_CHECK();
        from_zero = false;
        int j = 0;
        while (j < steps) {
            double *Wc = (j & 1) ? W1 : W0, *Wn = (j & 1) ? W0 : W1;
            hipLaunchKernelGGL((k_gm_arnoldi<Op, kPc>), dim3(g), dim3(kBlock), 0, s, A, V, n,
                               (const double *)Wc, Wn, j, ph0, (const GmState *)st);
            hipLaunchKernelGGL(k_gm_fold_h, dim3(j + 1), dim3(kBlock), 0, s, (const double *)ph0, g,
                               j, st, 0);
            hipLaunchKernelGGL((k_gm_cgs<Op>), dim3(g), dim3(kBlock), 0, s, A, (const double *)V, n,
                               Wn, j, ph0, (const GmState *)st, 0);
            hipLaunchKernelGGL(k_gm_fold_h, dim3(j + 1), dim3(kBlock), 0, s, (const double *)ph0, g,
                               j, st, 1);
            hipLaunchKernelGGL((k_gm_cgs<Op>), dim3(g), dim3(kBlock), 0, s, A, (const double *)V, n,
                               Wn, j, pn, (const GmState *)st, 1);
            hipLaunchKernelGGL(k_gm_fold_n, dim3(1), dim3(kBlock), 0, s, (const double *)pn, g,
                               j + 1, st);
            LAUNCH_CHECK();
            ++j;
            if (j % check == 0 && j < steps) {
                HIP_TRY(hipMemcpyAsync(c->hdone, &st->done, sizeof(int32_t), hipMemcpyDeviceToHost, s));
                LCS_TRY(wait_for(c, s));
                if (c->hdone[0]) break;
            }
        }
        hipLaunchKernelGGL(k_gm_finish, dim3(1), dim3(kBlock), 0, s, st);
        hipLaunchKernelGGL((k_gm_update<Op, kPc>), dim3(g), dim3(kBlock), 0, s, A, (const double *)V,
                           n, x, (const GmState *)st);
        LAUNCH_CHECK();
        HIP_TRY(hipMemcpyAsync(c->hgm, st, sizeof(GmState), hipMemcpyDeviceToHost, s));
        LCS_TRY(wait_for(c, s));
        const GmState &h = *c->hgm;
        out->its += h.k;
        if (h.status != kStOk) return status_of(h.status);
        if (h.done || out->its >= o->max_iter) {
            LCS_TRY(launch_resnorm(c, A, rhs, (const double *)x, (double *)nullptr, tol_base,
                                   tol_factor, s));
            LCS_TRY(read_scalars(c, s));
            out->rr = c->hsc->res.rr;
            if (c->hsc->res.status != kStOk) return status_of(c->hsc->res.status);
            if (c->hsc->res.done) return LCS_OK;
            if (out->its >= o->max_iter || outer >= o->max_outer) return status_of(kStNoConv);
            ++outer;
            out->n_outer += 1;
        }
    }
}

template <class Op>
lcs_status run_gmres(lcs_ctx *c, const Op &A, const double *rhs, double *x, bool x_zero,
                     const double *tol_base, double tol_factor, const lcs_options *o, hipStream_t s,
                     SolveOut *out) {
    *out = SolveOut();
    if (A.units() == 0) return LCS_OK;
    if (o->precond == LCS_PC_JACOBI)
        return run_gmres_t<Op, 1>(c, A, rhs, x, x_zero, tol_base, tol_factor, o, s, out);
    return run_gmres_t<Op, 0>(c, A, rhs, x, x_zero, tol_base, tol_factor, o, s, out);
}

// Solve op x = rhs: GMRES for a non-symmetric operator (the full-storage
// stencil at compile time, the restricted system of one at run time), else
// PCG as above.
template <class Op64, class Op32>
lcs_status solve_system(lcs_ctx *c, const Op64 &A, const Op32 &A32, int ncol, const double *rhs,
                        double *x, bool x_zero, const double *tol_base, double tol_factor,
                        const lcs_options *o, hipStream_t s, SolveOut *out, int scope,
                        bool gmres = false) {
    if constexpr (is_nonsym<Op64>) {
        return run_gmres(c, A, rhs, x, x_zero, tol_base, tol_factor, o, s, out);
    } else {
        if constexpr (is_ell<Op64>) {
            if (gmres) return run_gmres(c, A, rhs, x, x_zero, tol_base, tol_factor, o, s, out);
        }
        return solve_system_sym(c, A, A32, ncol, rhs, x, x_zero, tol_base, tol_factor, o, s, out,
                                scope);
    }
}
// ---------------------------------------------------------------------------
// Algorithm 2 / Algorithm 3: scores, threshold, expansion, compaction
// ---------------------------------------------------------------------------
// Neighbourhood of a structured stencil for k_expand_w: 5 (2-D cross),
// 9 (2-D 3 x 3), 7 (3-D cross); 0: general sparse rows (k_expand).
template <class SOp>
struct expand_shape : std::integral_constant<int, 0> {};
template <>
struct expand_shape<Stencil5<double>> : std::integral_constant<int, 5> {};
template <>
struct expand_shape<Stencil9<double>> : std::integral_constant<int, 9> {};
template <>
struct expand_shape<Stencil9N<double>> : std::integral_constant<int, 9> {};
template <>
struct expand_shape<Stencil7<double>> : std::integral_constant<int, 7> {};

// Scalar operators whose restricted systems may take the short column form
// (UEllShort): the symmetric 2-D stencils.
template <class SOp>
struct short_cols_ok : std::false_type {};
template <>
struct short_cols_ok<Stencil5<double>> : std::true_type {};
template <>
struct short_cols_ok<Stencil9<double>> : std::true_type {};
// ... and whose red-black colour-blocked restricted systems may take the
// red-black row codes (UEllRB): the five- and seven-point stencils
template <class SOp>
struct rb_code_ok : std::false_type {};
template <>
struct rb_code_ok<Stencil5<double>> : std::true_type {};
template <>
struct rb_code_ok<Stencil7<double>> : std::true_type {};

// Leaves s (r^(0) or g) in B_SCORE, stamps in B_STAMP, inv in B_INV and the
// ascending domain in idx; returns K (host).  eps0 >= 0: ||b|| (from the
// score pass) goes to dsc->bnorm, and an x0 with ||b - A x0|| <= eps0 ||b||
// gives the empty domain and hsc->ms.conv0 = 1.  xcopy (optional): the score
// pass also copies x0 there.
template <class SOp, class UOp>
lcs_status build_domain(lcs_ctx *c, const SOp &As, const UOp &Au, const double *b,
                        const double *x0, int mode, int thresh, double theta, int e_max,
                        double eps0, int32_t *idx, int64_t *K, hipStream_t s,
                        double *xcopy = nullptr) {
    const int64_t n = As.n;
    const Tiling T = tiling_for(n);
    const int gs = grid_for(Au, kRedGrid);
    double *score;
    uint8_t *stamp;
    int32_t *inv, *blockoff;
    LCS_TRY(get_buf(c, B_SCORE, n, &score));
    LCS_TRY(get_buf(c, B_STAMP, T.npad, &stamp));
    LCS_TRY(get_buf(c, B_INV, n, &inv));
    LCS_TRY(get_buf(c, B_BLOCKOFF, 2 * kMaxGrid, &blockoff));
    const bool timed = c->prof_what == LCS_TIME_SCORE;
    if (mode == LCS_MODE_RESIDUAL)
        LCS_TRY(launch_maybe_timed(c, timed, k_score<UOp, 0>, gs, s, Au, b, x0, score,
                                   slot(c, kPtScore), xcopy));
    else
        LCS_TRY(launch_maybe_timed(c, timed, k_score<UOp, 1>, gs, s, Au, b, x0, score,
                                   slot(c, kPtScore), xcopy));
    const int gmark = (int)std::min<int64_t>(T.npad / kTile, 2048);   // 2048 stamps per block step
    hipLaunchKernelGGL(k_mark, dim3(gmark), dim3(kBlock), 0, s, (const double *)score, stamp, n,
                       T.npad, thresh, theta, eps0, (const double *)slot(c, kPtScore), gs, c->dsc);
    LAUNCH_CHECK();
    const int ex = mode == LCS_MODE_RESIDUAL ? e_max : 0;
    const Launch Le = dims_wide(n, 4096);   // one partial per block
    constexpr int shape = expand_shape<SOp>::value;
    for (int m = 1; m <= ex; ++m) {
        const double *prev = slot(c, kPtExp0 + ((m - 1) & 1));
        double *cur = slot(c, kPtExp0 + (m & 1));
        if constexpr (shape != 0) {
            if (As.nx % 8 == 0) {   // eight cells per thread, rows of whole words
                const int64_t plane = shape == 7 ? (int64_t)As.nx * As.ny : 0;
                hipLaunchKernelGGL((k_expand_w<SOp, shape>), dim3(Le.grid), dim3(kBlock), 0, s, As,
                                   (const double *)score, x0, stamp, m, As.nx, plane, prev, cur,
                                   c->dsc);
                continue;
            }
        }
        hipLaunchKernelGGL((k_expand<SOp>), dim3(Le.grid), dim3(kBlock), 0, s, As,
                           (const double *)score, x0, stamp, m, Le.chunk, prev, cur, c->dsc);
    }
    LAUNCH_CHECK();
    hipLaunchKernelGGL(k_count, dim3(T.grid), dim3(kBlock), 0, s, (const uint8_t *)stamp, T.ntiles,
                       T.tiles_per_block, blockoff, ex, (const double *)slot(c, kPtExp0 + (ex & 1)),
                       Le.grid, c->dsc);
    hipLaunchKernelGGL(k_scatter, dim3(T.grid), dim3(kBlock), 0, s, (const uint8_t *)stamp, n,
                       T.ntiles, T.tiles_per_block, (const int32_t *)blockoff, idx, inv, c->dsc);
    LAUNCH_CHECK();
    LCS_TRY(read_scalars(c, s));
    *K = c->hsc->ms.K;
    return LCS_OK;
}

// ---------------------------------------------------------------------------
// restricted system and local solve (steps 3-7 of Algorithm 1)
// ---------------------------------------------------------------------------
template <int W>
struct Restricted {
    UEll<double, W> B64;
    UEll<float, W> B32;
    double *rhs;
    bool row_coded;   // B64 / B32 in UEllShort's form (code), their col unset
    RowCode code;
    bool rb_coded;    // B64 / B32 in UEllRB's form (rbcode), their col unset
    RBCode rbcode;
};
template <int W>
UEllShort<double, W> short64(const Restricted<W> &R) { return {R.B64, R.code}; }
template <int W>
UEllShort<float, W> short32(const Restricted<W> &R) { return {R.B32, R.code}; }
template <int W>
UEllRB<double, W> rb64(const Restricted<W> &R) { return {R.B64, R.rbcode}; }
template <int W>
UEllRB<float, W> rb32(const Restricted<W> &R) { return {R.B32, R.rbcode}; }

// UEllRB's code arrays in the column buffer of a K-row system (13 K bytes
// of its 4 W K): the distance words, then q, then the presence bits.
RBCode rb_code_in(int32_t *col, int64_t K) {
    uint64_t *d = reinterpret_cast<uint64_t *>(col);
    int32_t *q = reinterpret_cast<int32_t *>(d + K);
    return RBCode{d, q, reinterpret_cast<uint8_t *>(q + K)};
}

// B = A[idx, idx] in ELL (one pass, no scan); rhs = r[idx] when r is given.
// short_cols: in UEllShort's form (the caller checks that the domain is in
// grid order on a five- or nine-point stencil whose reach fits), its row
// codes in the column buffer.  rb_code: in UEllRB's form (the caller checks
// that idx is the red-black blocked order on a five- or seven-point stencil
// whose reach fits, and k_cblk_place left each row's q at the start of the
// column buffer).
template <int W, class SOp>
lcs_status gather(lcs_ctx *c, const SOp &A, const int32_t *idx, int64_t K, const int32_t *inv,
                  const double *r, bool with32, bool short_cols, Restricted<W> *R, hipStream_t s,
                  bool rb_code = false) {
    int32_t *col;
    double *val, *dg, *rhs;
    float *val32 = nullptr, *dg32 = nullptr;
    uint8_t *clr;
    LCS_TRY(get_buf(c, B_COL, (size_t)K * W, &col));
    LCS_TRY(get_buf(c, B_VAL, (size_t)K * W, &val));
    LCS_TRY(get_buf(c, B_DG, K, &dg));
    LCS_TRY(get_buf(c, B_CLR, K, &clr));
    LCS_TRY(get_buf(c, B_RHSL, K, &rhs));
    if (with32) {
        LCS_TRY(get_buf(c, B_VAL32, (size_t)K * W, &val32));
        LCS_TRY(get_buf(c, B_DG32, K, &dg32));
    }
    R->row_coded = false;
    R->code = RowCode{nullptr, nullptr};
    R->rb_coded = false;
    R->rbcode = RBCode{nullptr, nullptr, nullptr};
    if constexpr (rb_code_ok<SOp>::value) {
        if (rb_code) {
            static_assert(SOp::kSlots == W, "row codes take the stencil's slots");
            const RBCode rc = rb_code_in(col, K);
            hipLaunchKernelGGL((k_gather_rbcode<SOp>), dim3(flat_grid(K)), dim3(kBlock), 0, s, A,
                               idx, K, inv, rc.q, const_cast<uint64_t *>(rc.d),
                               const_cast<uint8_t *>(rc.mask), val, val32, dg, dg32, clr, r,
                               r ? rhs : nullptr);
            LAUNCH_CHECK();
            R->B64 = {nullptr, val, dg, clr, K};
            R->B32 = {nullptr, val32, dg32, clr, K};
            R->rhs = rhs;
            R->rb_coded = true;
            R->rbcode = rc;
            return LCS_OK;
        }
    }
    if (rb_code) return fail(LCS_EINVAL, "red-black row codes on this operator");
    if constexpr (short_cols_ok<SOp>::value) {
        if (short_cols) {
            static_assert(SOp::kSlots == W, "row codes take the stencil's slots");
            // 5 bytes per row of the column buffer's 4 W
            uint32_t *of = reinterpret_cast<uint32_t *>(col);
            uint8_t *mk = reinterpret_cast<uint8_t *>(of + K);
            hipLaunchKernelGGL((k_gather_rowcode<SOp>), dim3(flat_grid(K)), dim3(kBlock), 0, s, A,
                               idx, K, inv, of, mk, val, val32, dg, dg32, clr, r,
                               r ? rhs : nullptr);
            LAUNCH_CHECK();
            R->B64 = {nullptr, val, dg, clr, K};
            R->B32 = {nullptr, val32, dg32, clr, K};
            R->rhs = rhs;
            R->row_coded = true;
            R->code = RowCode{of, mk};
            return LCS_OK;
        }
    }
    if (short_cols) return fail(LCS_EINVAL, "short column form on this operator");
    hipLaunchKernelGGL((k_gather_ell<SOp>), dim3(flat_grid(K)), dim3(kBlock), 0, s, A, idx, K, inv,
                       W, col, val, val32, dg, dg32, clr, r, r ? rhs : nullptr);
    LAUNCH_CHECK();
    R->B64 = {col, val, dg, clr, K};
    R->B32 = {col, val32, dg32, clr, K};
    R->rhs = rhs;
    return LCS_OK;
}

struct Timers {
    lcs_ctx *c;
    hipStream_t s;
    bool on;
    lcs_status mark(int k) {
        if (on) HIP_TRY(hipEventRecord(c->ev[k], s));
        return LCS_OK;
    }
    double ms(int a, int b) {
        if (!on) return 0.0;
        float v = 0.f;
        if (hipEventElapsedTime(&v, c->ev[a], c->ev[b]) != hipSuccess) {
            (void)hipGetLastError();
            return 0.0;
        }
        return v;
    }
};

template <class T>
struct is_pair9 : std::false_type {};
template <int W>
struct is_pair9<U9<double, 2, W>> : std::true_type {};

// Waves of `kernel` that the GPU holds at once: blocks per compute unit at
// its occupancy x compute units x 4; asked of the runtime once and kept in
// `cache`.
template <class K>
lcs_status resident_waves(K kernel, std::atomic<int64_t> &cache, int64_t *out) {
    int64_t v = cache.load();
    if (v == 0) {
        int nb = 0, cus = 0, dev = 0;
        HIP_TRY(hipGetDevice(&dev));
        HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
        HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kernel, kBlock, 0));
        v = std::max<int64_t>(1, (int64_t)nb * cus) * kWaves;
        cache.store(v);
    }
    *out = v;
    return LCS_OK;
}

// n_sweeps colour-ordered Gauss-Seidel sweeps on A x = b (Algorithm 1 step
// 7): one kernel per colour, or, for the nine-point stencil in strips of two
// cells, one kernel per pair of colours (k_gs_pair9: rows of one parity)
// through a second buffer.  With crit_eps >= 0 the nine-point path also
// forms the criterion of step 8 (||b - A x|| <= crit_eps ||b||, into
// dsc->res) in its last pass and sets *crit_done; other paths leave it to
// the caller.
// Whether launch_sweeps takes the one-pass path (k_gs_sweep9): the
// nine-point stencil in strips of two cells, four colours, with the
// criterion, on grids of at least kMaxGrid tiles of 16 rows.
template <class UOp>
bool one_pass_sweeps(const UOp &Au, int ncol, int n_sweeps, double crit_eps) {
    if constexpr (is_pair9<UOp>::value) {
        const int64_t strips1 = ((int64_t)Au.nx / 2 + kSweepOwn - 1) / kSweepOwn;
        return ncol == 4 && crit_eps >= 0.0 && n_sweeps > 0 &&
               strips1 * ((Au.ny + 15) / 16) >= kMaxGrid;
    } else {
        return false;
    }
}

template <class UOp>
lcs_status launch_sweeps(lcs_ctx *c, const UOp &Au, const double *b, double *x, int ncol,
                         int n_sweeps, hipStream_t s, double crit_eps = -1.0,
                         bool *crit_done = nullptr, bool tmp_holds_x = false) {
    const bool timed = c->prof_what == LCS_TIME_SMOOTH;
    if constexpr (is_pair9<UOp>::value) {
        if (ncol == 4) {
            double *tmp;
            LCS_TRY(get_buf(c, B_GSX, (size_t)Au.n, &tmp));
            const bool fuse = crit_eps >= 0.0 && n_sweeps > 0;
            const int64_t strips1 = ((int64_t)Au.nx / 2 + kSweepOwn - 1) / kSweepOwn;
            if (one_pass_sweeps(Au, ncol, n_sweeps, crit_eps)) {
                // Whole sweeps in one pass each (k_gs_sweep9), the last one
                // forming the criterion; they alternate between x and the
                // second buffer and end in x: an odd count starts from the
                // second buffer when it holds x already (tmp_holds_x), else
                // a copy brings the result back.  Tiles of an even number of
                // rows, at least 16 (a tile updates two or three rows
                // outside it again), grown until there is at most one per
                // wave that the GPU holds at once
                // (the kernel's occupancy, asked of the runtime once), so
                // that no wave waits for a second round; at most kMaxGrid
                // blocks (the partials).  Used once the grid has at least
                // kMaxGrid such tiles.
                static std::atomic<int64_t> held{0};
                int64_t waves = 0;
                LCS_TRY(resident_waves(k_gs_sweep9<UOp, true>, held, &waves));
                waves = std::min<int64_t>(waves, (int64_t)kMaxGrid * kWaves);
                int mh = 16;
                while (mh < Au.ny && strips1 * ((Au.ny + mh - 1) / mh) > waves) mh += 2;
                const int64_t tiles = strips1 * ((Au.ny + mh - 1) / mh);
                int grid = (int)std::min<int64_t>(kMaxGrid, (tiles + kWaves - 1) / kWaves);
                grid = std::min(kMaxGrid, std::max(kXcds, (grid + kXcds - 1) / kXcds * kXcds));
                const bool from_tmp = tmp_holds_x && (n_sweeps & 1);
                const double *src = from_tmp ? tmp : x;
                double *dst = from_tmp ? x : tmp;
                for (int sw = 0; sw < n_sweeps; ++sw) {
                    if (sw == n_sweeps - 1) {
                        LCS_TRY(launch_maybe_timed(c, timed, k_gs_sweep9<UOp, true>, grid, s, Au, b,
                                                   src, dst, mh, slot(c, kPtRes)));
                        hipLaunchKernelGGL(k_fin_res, dim3(1), dim3(kBlock), 0, s,
                                           (const double *)slot(c, kPtRes), grid,
                                           (const double *)&c->dsc->bnorm, crit_eps, c->dsc);
                        LAUNCH_CHECK();
                    } else {
                        LCS_TRY(launch_maybe_timed(c, timed, k_gs_sweep9<UOp, false>, grid, s, Au,
                                                   b, src, dst, mh, slot(c, kPtRes)));
                    }
                    src = dst;
                    dst = dst == tmp ? x : tmp;
                }
                if (src != x)
                    HIP_TRY(hipMemcpyAsync(x, src, sizeof(double) * (size_t)Au.n,
                                           hipMemcpyDeviceToDevice, s));
                *crit_done = true;
                return LCS_OK;
            }
            // two passes per sweep (k_gs_pair9), each over the rows of one
            // parity, in tiles of up to 32 rows, about 4096 of them on large
            // grids; with the criterion, the last pass forms it
            // (k_gs_pair9_res: 62 owned strips per wave, at most kMaxGrid
            // blocks, tiles grown to at most one per resident wave)
            const int64_t strips = ((int64_t)Au.nx / 2 + kPairStep - 1) / kPairStep;
            const int mh = (int)std::max<int64_t>(2, std::min<int64_t>(32, strips * Au.ny / 4096));
            const int64_t tiles = strips * ((Au.ny + mh - 1) / mh);
            int grid = (int)std::min<int64_t>(kStreamGrid, (tiles + kWaves - 1) / kWaves);
            grid = std::max(kXcds, (grid + kXcds - 1) / kXcds * kXcds);
            int mh_r = mh, grid_r = kXcds;
            if (fuse) {
                static std::atomic<int64_t> held_r{0};
                int64_t waves_r = 0;
                LCS_TRY(resident_waves(k_gs_pair9_res<UOp>, held_r, &waves_r));
                waves_r = std::min<int64_t>(waves_r, (int64_t)kMaxGrid * kWaves);
                const int64_t strips_r = ((int64_t)Au.nx / 2 + kPairOwn - 1) / kPairOwn;
                while (mh_r < Au.ny && strips_r * ((Au.ny + mh_r - 1) / mh_r) > waves_r) ++mh_r;
                const int64_t tiles_r = strips_r * ((Au.ny + mh_r - 1) / mh_r);
                grid_r = (int)std::min<int64_t>(kMaxGrid, (tiles_r + kWaves - 1) / kWaves);
                grid_r = std::min(kMaxGrid, std::max(kXcds, (grid_r + kXcds - 1) / kXcds * kXcds));
            }
            for (int sw = 0; sw < n_sweeps; ++sw) {
                LCS_TRY(launch_maybe_timed(c, timed, k_gs_pair9<UOp>, grid, s, Au, b,
                                           (const double *)x, tmp, 0, mh));
                if (fuse && sw == n_sweeps - 1) {
                    LCS_TRY(launch_maybe_timed(c, timed, k_gs_pair9_res<UOp>, grid_r, s, Au, b,
                                               (const double *)tmp, x, 1, mh_r, slot(c, kPtRes)));
                    hipLaunchKernelGGL(k_fin_res, dim3(1), dim3(kBlock), 0, s,
                                       (const double *)slot(c, kPtRes), grid_r,
                                       (const double *)&c->dsc->bnorm, crit_eps, c->dsc);
                    LAUNCH_CHECK();
                    *crit_done = true;
                } else {
                    LCS_TRY(launch_maybe_timed(c, timed, k_gs_pair9<UOp>, grid, s, Au, b,
                                               (const double *)tmp, x, 1, mh));
                }
            }
            return LCS_OK;
        }
    }
    const int grid = grid_for(Au, kStreamGrid);
    for (int sw = 0; sw < n_sweeps; ++sw)
        for (int col = 0; col < ncol; ++col)
            LCS_TRY(launch_maybe_timed(c, timed, k_gs_half<UOp, false>, grid, s, Au, b, x, col,
                                       (const Scalars *)nullptr, (double *)nullptr));
    return LCS_OK;
}

// x <- x + d on Omega after solving B d = r^(0)_Omega, then smoothing.
// r0: r^(0) over the whole grid when the caller already has it, else null.
// xcopy: the sweeps' second buffer when it holds a copy of x (kept equal to
// x through the update), else null.
template <int W, class SOp, class UOp>
lcs_status local_phase(lcs_ctx *c, const lcs_matrix *M, const SOp &As, const UOp &Au,
                       const double *b, double *x, const int32_t *idx, int64_t K,
                       const int32_t *inv, const double *r0, const lcs_options *o,
                       lcs_stats *st, Timers &tm, hipStream_t s, bool *crit_done,
                       double *xcopy = nullptr) {
    const int ncol = colours_of(M);
    if (K > 0) {
        if (!r0) {
            double *r;
            LCS_TRY(get_buf(c, B_SCORE, As.n, &r));
            LCS_TRY(launch_resnorm(c, Au, b, (const double *)x, r, &c->dsc->bnorm, o->eps, s));
            r0 = r;
        }
        // With the Gauss-Seidel preconditioner the rows of B go colour by
        // colour (ascending inside each colour, slots still in ascending
        // grid order): every row's arithmetic is unchanged, and a half sweep
        // reads its own colour's rows only.
        const int32_t *dom = idx;
        bool rb_code = false;
        struct ClearBlocks {
            lcs_ctx *c;
            ~ClearBlocks() { c->cblk.n = 0; }
        } clear_blocks{c};
        if (c->colour_blocks && o->precond == LCS_PC_RBSGS && ncol >= 2 && ncol <= kMaxBlkColours &&
            !uses_gmres(M)) {
            int32_t *idxb, *cnt;
            LCS_TRY(get_buf(c, B_IDXB, K, &idxb));
            LCS_TRY(get_buf(c, B_CBLK, (size_t)kMaxBlkColours * kMaxGrid, &cnt));
            // red-black rows coded per row: each row's q straight into the
            // code's place in the column buffer
            int32_t *qv = nullptr;
            rb_code = rb_code_ok<SOp>::value && c->short_cols && ncol == 2 &&
                      stencil_reach(M) <= kMaxRB16;
            if (rb_code) {
                int32_t *colbuf;
                LCS_TRY(get_buf(c, B_COL, (size_t)K * W, &colbuf));
                qv = const_cast<int32_t *>(rb_code_in(colbuf, K).q);
            }
            const int g = (int)std::min<int64_t>(kMaxGrid, std::max<int64_t>(1, (K + 2047) / 2048));
            const int64_t chunk = (K + g - 1) / g;
            hipLaunchKernelGGL((k_cblk_count<SOp>), dim3(g), dim3(kBlock), 0, s, As, idx, K, chunk,
                               ncol, cnt);
            hipLaunchKernelGGL((k_cblk_place<SOp>), dim3(g), dim3(kBlock), 0, s, As, idx, K, chunk,
                               ncol, (const int32_t *)cnt, idxb, const_cast<int32_t *>(inv), c->dsc,
                               qv);
            LAUNCH_CHECK();
            LCS_TRY(read_scalars(c, s));
            if (c->hsc->cstart[ncol] != K) return fail(LCS_EHIP, "colour blocks do not cover the domain");
            c->cblk.n = ncol;
            for (int q = 0; q <= ncol; ++q) c->cblk.start[q] = c->hsc->cstart[q];
            dom = idxb;
        }
        // a domain in grid order keeps every column within the stencil's
        // reach of its row (the short form is built for the symmetric 2-D
        // stencils)
        const bool short_cols = short_cols_ok<SOp>::value && c->short_cols && dom == idx &&
                                stencil_reach(M) <= kMaxCol16;
        Restricted<W> R;
        LCS_TRY(gather<W>(c, As, dom, K, inv, r0, o->precision == LCS_PREC_MIXED, short_cols, &R,
                          s, rb_code));
        double *d;
        LCS_TRY(get_buf(c, B_DL, K, &d));
        const double tl = o->tol_local > 0 ? o->tol_local : o->eps;
        SolveOut so;
        lcs_status ls = LCS_OK;
        bool solved = false;
        if constexpr (short_cols_ok<SOp>::value) {
            if (R.row_coded) {
                ls = solve_system(c, short64(R), short32(R), ncol, (const double *)R.rhs, d,
                                  true, &c->dsc->bnorm, tl, o, s, &so, 1, uses_gmres(M));
                solved = true;
            }
        }
        if constexpr (rb_code_ok<SOp>::value) {
            if (!solved && R.rb_coded) {
                ls = solve_system(c, rb64(R), rb32(R), ncol, (const double *)R.rhs, d, true,
                                  &c->dsc->bnorm, tl, o, s, &so, 1, uses_gmres(M));
                solved = true;
            }
        }
        if (!solved)
            ls = solve_system(c, R.B64, R.B32, ncol, (const double *)R.rhs, d, true,
                              &c->dsc->bnorm, tl, o, s, &so, 1, uses_gmres(M));
        // a local solve that stops at its iteration cap still improves x;
        // the global finish takes over from there
        if (ls != LCS_OK && ls != LCS_ENOCONV) return ls;
        st->its_local = so.its;   // -1: read from the device state after the next sync
        st->n_outer += so.n_outer;
        hipLaunchKernelGGL(k_scatter_add, dim3(flat_grid(K)), dim3(kBlock), 0, s, dom,
                           (const double *)d, K, x, xcopy);
        LAUNCH_CHECK();
    }
    LCS_TRY(tm.mark(2));
    *crit_done = false;
    if (o->n_smooth > 0)
        LCS_TRY(launch_sweeps(c, Au, b, x, ncol, o->n_smooth, s, o->eps, crit_done,
                              xcopy != nullptr));
    LCS_TRY(tm.mark(3));
    return LCS_OK;
}

// inv for a caller-supplied domain; rejects indices out of range or not
// strictly ascending before anything reads through them.
lcs_status set_inv(lcs_ctx *c, const int32_t *idx, int64_t K, int64_t n, int32_t *inv,
                   hipStream_t s) {
    hipLaunchKernelGGL(k_fill<int32_t>, dim3(1), dim3(1), 0, s, &c->dsc->bad_idx, 0, (int64_t)1);
    hipLaunchKernelGGL(k_fill<int32_t>, dim3(flat_grid(n)), dim3(kBlock), 0, s, inv, -1, n);
    if (K > 0)
        hipLaunchKernelGGL(k_set_inv, dim3(flat_grid(K)), dim3(kBlock), 0, s, idx, K, n, inv, c->dsc);
    LAUNCH_CHECK();
    LCS_TRY(read_scalars(c, s));
    if (c->hsc->bad_idx) return fail(LCS_EINVAL, "idx must be strictly ascending indices in [0, N)");
    return LCS_OK;
}

// After a sync: the local PCG outcome left on the device (FP64 path).
lcs_status finish_local(lcs_ctx *c, lcs_stats *st) {
    if (st->its_local >= 0) return LCS_OK;
    st->its_local = c->hsc->saved_it[1];
    c->last_its[1][0] = st->its_local;
    const int ls = c->hsc->saved_status[1];
    if (ls == kStBreakdown || ls == kStNonFinite) return status_of(ls);
    return LCS_OK;
}

void init_stats(lcs_stats *st) {
    std::memset(st, 0, sizeof(*st));
    st->relres_after_local = NAN;
    st->relres_final = NAN;
}

bool vec_ok(std::initializer_list<const void *> ps) {
    for (const void *p : ps)
        if (!aligned16(p)) return false;
    return true;
}

lcs_status check_mode(int32_t mode, int32_t thresh_kind, double theta, int32_t e_max) {
    if (mode != LCS_MODE_RESIDUAL && mode != LCS_MODE_GRADIENT) return fail(LCS_EINVAL, "mode");
    if (thresh_kind < 0 || thresh_kind > 2) return fail(LCS_EINVAL, "threshold kind");
    if (thresh_kind == LCS_THRESH_PAPER && mode != LCS_MODE_RESIDUAL)
        return fail(LCS_EINVAL, "the paper threshold belongs to the residual mode");
    if (e_max < 0 || e_max > 250) return fail(LCS_EINVAL, "e_max must be in 0..250");
    if (!(theta >= 0.0)) return fail(LCS_EINVAL, "theta must be >= 0");
    return LCS_OK;
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================
// ---------------------------------------------------------------------------
// batched solves (G systems on one grid, one workgroup each)
// ---------------------------------------------------------------------------
namespace {

template <class S>
lcs_status launch_batch(lcs_ctx *c, const S &A, int pc, const BatchArgs &a, int32_t G,
                        const double *b, double *x, double *ws, uint8_t *stamp, int32_t *idx,
                        BatchOut *out, hipStream_t s) {
    // systems of at most kLdsRows cells keep PCG's p and q (GMRES: z and w)
    // in LDS
    const bool lds = A.n <= kLdsRows;
    if (pc == LCS_PC_JACOBI) {
        if (lds)
            hipLaunchKernelGGL((k_batch_solve<S, 1, true>), dim3(G), dim3(kBatchBlock), 0, s, A, a, b,
                               x, ws, stamp, idx, out);
        else
            hipLaunchKernelGGL((k_batch_solve<S, 1, false>), dim3(G), dim3(kBatchBlock), 0, s, A, a, b,
                               x, ws, stamp, idx, out);
    } else {
        if (lds)
            hipLaunchKernelGGL((k_batch_solve<S, 0, true>), dim3(G), dim3(kBatchBlock), 0, s, A, a, b,
                               x, ws, stamp, idx, out);
        else
            hipLaunchKernelGGL((k_batch_solve<S, 0, false>), dim3(G), dim3(kBatchBlock), 0, s, A, a, b,
                               x, ws, stamp, idx, out);
    }
    LAUNCH_CHECK();
    return LCS_OK;
}

lcs_status solve_batched(lcs_ctx *c, const lcs_matrix *A, int32_t G, const double *b, double *x,
                         int local, int32_t mode, int32_t thresh_kind, double theta, int32_t e_max,
                         const lcs_options *o, lcs_stats *st, void *stream) {
    if (!c) return fail(LCS_EINVAL, "ctx is NULL");
    LCS_TRY(check_matrix(A));
    if (A->kind == LCS_CSR) return fail(LCS_EINVAL, "batched solves take the stencil kinds");
    LCS_TRY(check_options_for(o, A));
    LCS_TRY(check_ptr(b, "b"));
    LCS_TRY(check_ptr(x, "x"));
    if (local) LCS_TRY(check_mode(mode, thresh_kind, theta, e_max));
    if (G < 1 || G > kMaxBatch) return fail(LCS_EINVAL, "batch size G must be 1..65535");
    if (o->precision != LCS_PREC_FP64) return fail(LCS_EINVAL, "batched solves run in FP64");
    if (o->precond == LCS_PC_RBSGS)
        return fail(LCS_EINVAL, "batched solves take the Jacobi preconditioner or none");
    const int64_t n = (int64_t)A->nx * A->ny * A->nz;
    if (n > kMaxBatchN) return fail(LCS_EINVAL, "batched solves take at most 2^24 cells per system");
    LCS_TRY(plan_call(c, A, o, kWhatBatch, G));
    hipStream_t s = (hipStream_t)stream;
    BatchArgs a{};
    a.coef_stride = (int64_t)n_arrays(A->kind) * n;
    a.local = local;
    a.mode = mode;
    a.thresh = thresh_kind;
    a.theta = theta;
    a.e_max = e_max;
    a.eps = o->eps;
    a.tol_local = o->tol_local > 0.0 ? o->tol_local : o->eps;
    a.max_iter = o->max_iter;
    a.max_outer = o->max_outer;
    a.n_smooth = o->n_smooth;
    a.restart = 0;
    a.gm_V = nullptr;
    if (A->kind == LCS_STENCIL9N_2D) {   // GMRES(m): one basis per system
        a.restart = o->restart;
        LCS_TRY(get_buf(c, B_BGMV, (size_t)(a.restart + 1) * n * G, &a.gm_V));
    }
    double *ws;
    uint8_t *stamp;
    int32_t *idx;
    BatchOut *dout;
    LCS_TRY(get_buf(c, B_BWS, (size_t)4 * n * G, &ws));
    LCS_TRY(get_buf(c, B_BSTAMP, (size_t)n * G, &stamp));
    LCS_TRY(get_buf(c, B_BIDX, (size_t)n * G, &idx));
    LCS_TRY(get_buf(c, B_BOUT, (size_t)G, &dout));
    switch (A->kind) {
    case LCS_STENCIL5_2D:
        LCS_TRY(launch_batch(c, sop5<double>(A, A->coef), o->precond, a, G, b, x, ws, stamp, idx, dout, s));
        break;
    case LCS_STENCIL9_2D:
        LCS_TRY(launch_batch(c, sop9<double>(A, A->coef), o->precond, a, G, b, x, ws, stamp, idx, dout, s));
        break;
    case LCS_STENCIL9N_2D:
        LCS_TRY(launch_batch(c, sop9n<double>(A, A->coef), o->precond, a, G, b, x, ws, stamp, idx, dout, s));
        break;
    default:
        LCS_TRY(launch_batch(c, sop7<double>(A, A->coef), o->precond, a, G, b, x, ws, stamp, idx, dout, s));
        break;
    }
    int first_bad = -1;
    int first_status = kStOk;
    for (int32_t g = 0; g < G; ++g) {
        const int slot_g = g % kBoutChunk;
        if (slot_g == 0) {   // the next chunk of results
            const int m = std::min<int32_t>(kBoutChunk, G - g);
            HIP_TRY(hipMemcpyAsync(c->hbout, dout + g, sizeof(BatchOut) * (size_t)m,
                                   hipMemcpyDeviceToHost, s));
            LCS_TRY(wait_for(c, s));
        }
        const BatchOut &r = c->hbout[slot_g];
        if (st) {
            init_stats(&st[g]);
            st[g].K = r.K;
            st[g].e_rounds = r.e_rounds;
            st[g].its_local = r.its_local;
            st[g].its_global = r.its_global;
            st[g].n_outer = r.n_outer;
            st[g].tau = r.tau;
            if (local) st[g].relres_after_local = r.relres_after_local;
            st[g].relres_final = r.relres_final;
        }
        if (r.status != kStOk && first_bad < 0) {
            first_bad = g;
            first_status = r.status;
        }
    }
    if (first_bad >= 0) {
        const lcs_status e = status_of(first_status);
        return fail(e, "system " + std::to_string(first_bad) + " of the batch: " + g_err);
    }
    return LCS_OK;
}

// Context creation: device state and partials from ws (caller-owned, at
// least ws_head_bytes()) or from hipMalloc (ws == NULL); pinned host copies
// and events in both cases.
lcs_status create_ctx(lcs_ctx **out, void *ws, size_t ws_bytes) {
    if (!out) return fail(LCS_EINVAL, "ctx is NULL");
    *out = nullptr;
    lcs_ctx *c = new lcs_ctx();
    auto cleanup = [&](lcs_status st) {
        lcs_destroy(c);
        return st;
    };
    if (hipGetDevice(&c->device) != hipSuccess) return cleanup(fail(LCS_EHIP, "no HIP device"));
    if (ws) {
        c->ws = static_cast<char *>(ws);
        c->ws_bytes = ws_bytes;
        c->dsc = reinterpret_cast<Scalars *>(c->ws);
        c->partials = reinterpret_cast<double *>(c->ws + align_up(sizeof(Scalars)));
    } else {
        if (hipMalloc(&c->dsc, sizeof(Scalars)) != hipSuccess) return cleanup(fail(LCS_ENOMEM, "state"));
        if (hipMalloc(&c->partials, sizeof(double) * kSlotElems * kPtSlots) != hipSuccess)
            return cleanup(fail(LCS_ENOMEM, "partials"));
    }
    if (hipMemset(c->dsc, 0, sizeof(Scalars)) != hipSuccess) return cleanup(fail(LCS_EHIP, "memset"));
    if (hipHostMalloc(&c->hsc, sizeof(Scalars), hipHostMallocDefault) != hipSuccess)
        return cleanup(fail(LCS_ENOMEM, "pinned state"));
    if (hipHostMalloc(&c->hdone, 2 * sizeof(int32_t), hipHostMallocDefault) != hipSuccess)
        return cleanup(fail(LCS_ENOMEM, "pinned flags"));
    if (hipHostMalloc(&c->hpcg, 2 * sizeof(PcgState), hipHostMallocDefault) != hipSuccess)
        return cleanup(fail(LCS_ENOMEM, "pinned PCG state"));
    if (hipHostMalloc(&c->hgm, sizeof(GmState), hipHostMallocDefault) != hipSuccess)
        return cleanup(fail(LCS_ENOMEM, "pinned GMRES state"));
    if (hipHostMalloc(&c->hbout, sizeof(BatchOut) * kBoutChunk, hipHostMallocDefault) != hipSuccess)
        return cleanup(fail(LCS_ENOMEM, "pinned batch results"));
    for (auto &e : c->ev)
        if (hipEventCreate(&e) != hipSuccess) return cleanup(fail(LCS_EHIP, "event"));
    for (auto &e : c->chk)
        if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess)
            return cleanup(fail(LCS_EHIP, "event"));
    if (hipEventCreateWithFlags(&c->done_ev, hipEventDisableTiming) != hipSuccess)
        return cleanup(fail(LCS_EHIP, "event"));
    if (hipDeviceSynchronize() != hipSuccess) return cleanup(fail(LCS_EHIP, "sync"));
    *out = c;
    return LCS_OK;
}
}  // namespace

// ---------------------------------------------------------------------------
// local domain without allocation: the scratch array
// ---------------------------------------------------------------------------
// Device state, partials and the domain's buffers (scores, stamps, inv,
// block counts) of lcs_build_local_domain_static, for grids of at most
// kStaticMaxN cells.  Each GPU the library runs on holds its own copy until
// the process ends.  Host code never passes `scratch` itself to a kernel (on
// the host it only names the symbol): static_scratch() looks up its device
// address once per device and every use goes through that address.
constexpr int64_t kStaticMaxN = int64_t(1) << 21;
constexpr size_t kStaticScratchBytes = size_t(28) << 20;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// Device address of the scratch array on the current device (looked up on
// the first call on each device, with that device current).
lcs_status static_scratch(void **out, int *device) {
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(LCS_EINVAL, "device index beyond 63");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return fail(LCS_EHIP, "hipGetSymbolAddress gave no address for the scratch array");
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    *device = dev;
    return LCS_OK;
}
}  // namespace

extern "C" {

void lcs_default_options(lcs_options *o) {
    if (!o) return;
    o->eps = 1e-10;
    o->tol_local = 0.0;
    o->inner_tol = 1e-5;
    o->max_iter = 20000;
    o->precond = LCS_PC_JACOBI;
    o->precision = LCS_PREC_FP64;
    o->n_smooth = 1;
    o->check_every = 8;
    o->max_outer = 10;
    o->restart = 40;
}

const char *lcs_last_error(void) { return g_err.c_str(); }

lcs_status lcs_create(lcs_ctx **out) { return create_ctx(out, nullptr, 0); }

lcs_status lcs_create_with_workspace(lcs_ctx **out, void *workspace, size_t bytes) {
    if (!out) return fail(LCS_EINVAL, "ctx is NULL");
    *out = nullptr;
    if (!workspace) return fail(LCS_EINVAL, "workspace is NULL");
    if ((uintptr_t)workspace % kWsAlign != 0)
        return fail(LCS_EINVAL, "workspace must be 256-byte aligned");
    if (bytes < ws_head_bytes())
        return fail(LCS_EINVAL, "workspace smaller than its fixed head of " +
                                    std::to_string(ws_head_bytes()) + " bytes");
    return create_ctx(out, workspace, bytes);
}

size_t lcs_workspace_bytes(const lcs_matrix *A, const lcs_options *o) {
    if (check_matrix(A) != LCS_OK) return 0;
    if (o && check_options_for(o, A) != LCS_OK) return 0;
    size_t m = 0;
    for (int what : {kWhatPiece, kWhatSpmv32, kWhatDomain, kWhatGather, kWhatSolve})
        m = std::max(m, plan_total(A, o, what, 0));
    return m;
}

size_t lcs_workspace_bytes_batched(const lcs_matrix *A, int32_t G, const lcs_options *o) {
    if (check_matrix(A) != LCS_OK) return 0;
    if (o && check_options_for(o, A) != LCS_OK) return 0;
    if (G < 1 || G > kMaxBatch) {
        fail(LCS_EINVAL, "batch size G must be 1..65535");
        return 0;
    }
    return plan_total(A, o, kWhatBatch, G);
}

void lcs_destroy(lcs_ctx *c) {
    if (!c) return;
    (void)hipDeviceSynchronize();
    for (int i = 0; i < B_NUM; ++i)
        if (c->buf[i]) (void)hipFree(c->buf[i]);
    if (!c->ws) {
        if (c->dsc) (void)hipFree(c->dsc);
        if (c->partials) (void)hipFree(c->partials);
    }
    if (c->hsc) (void)hipHostFree(c->hsc);
    if (c->hdone) (void)hipHostFree(c->hdone);
    if (c->hpcg) (void)hipHostFree(c->hpcg);
    if (c->hbout) (void)hipHostFree(c->hbout);
    if (c->hgm) (void)hipHostFree(c->hgm);
    for (auto &e : c->ev)
        if (e) (void)hipEventDestroy(e);
    for (auto &e : c->chk)
        if (e) (void)hipEventDestroy(e);
    if (c->done_ev) (void)hipEventDestroy(c->done_ev);
    for (auto &e : c->prof_ev) (void)hipEventDestroy(e);
    delete c;
}

lcs_status lcs_residual(lcs_ctx *c, const lcs_matrix *A, const double *b, const double *x,
                        double *r, void *stream) {
    if (!c) return fail(LCS_EINVAL, "ctx is NULL");
    LCS_TRY(check_matrix(A));
    LCS_TRY(plan_call(c, A, nullptr, kWhatPiece));
    LCS_TRY(prepare_matrix(c, A, (hipStream_t)stream));
    LCS_TRY(check_ptr(b, "b"));
    LCS_TRY(check_ptr(x, "x"));
    LCS_TRY(check_ptr(r, "r"));
    hipStream_t s = (hipStream_t)stream;
    return with_ops(c, A, nullptr, vec_ok({b, x, r}), [&](auto, auto op, auto, auto) -> lcs_status {
        const int64_t n = op.units() * decltype(op)::V;
        LCS_TRY(launch_norm(c, b, n, &c->dsc->bnorm, s));
        LCS_TRY(launch_resnorm(c, op, b, x, r, &c->dsc->bnorm, 1.0, s));
        LCS_TRY(wait_for(c, s));
        return LCS_OK;
    });
}

lcs_status lcs_gradient(lcs_ctx *c, const lcs_matrix *A, const double *x, double *g, void *stream) {
    if (!c) return fail(LCS_EINVAL, "ctx is NULL");
    LCS_TRY(check_matrix(A));
    LCS_TRY(plan_call(c, A, nullptr, kWhatPiece));
    LCS_TRY(prepare_matrix(c, A, (hipStream_t)stream));
    LCS_TRY(check_ptr(x, "x"));
    LCS_TRY(check_ptr(g, "g"));
    hipStream_t s = (hipStream_t)stream;
    return with_ops(c, A, nullptr, vec_ok({x, g}), [&](auto, auto op, auto, auto) -> lcs_status {
        const int grid = grid_for(op, kRedGrid);
        hipLaunchKernelGGL((k_score<decltype(op), 1>), dim3(grid), dim3(kBlock), 0, s, op, x, x, g,
                           slot(c, kPtScore), (double *)nullptr);
        LAUNCH_CHECK();
        LCS_TRY(wait_for(c, s));
        return LCS_OK;
    });
}

lcs_status lcs_spmv(lcs_ctx *c, const lcs_matrix *A, const void *x, void *y, int32_t precision,
                    int32_t reps, void *stream) {
    if (!c) return fail(LCS_EINVAL, "ctx is NULL");
    LCS_TRY(check_matrix(A));
    LCS_TRY(plan_call(c, A, nullptr, precision == LCS_PREC_MIXED ? kWhatSpmv32 : kWhatPiece));
    LCS_TRY(prepare_matrix(c, A, (hipStream_t)stream));
    LCS_TRY(check_ptr(x, "x"));
    LCS_TRY(check_ptr(y, "y"));
    if (precision != LCS_PREC_FP64 && precision != LCS_PREC_MIXED)
        return fail(LCS_EINVAL, "unknown precision");
    hipStream_t s = (hipStream_t)stream;
    const float *c32 = nullptr;
    LCS_TRY(ensure_coef32(c, A, precision == LCS_PREC_MIXED, &c32, s));
    return with_ops(c, A, c32, vec_ok({x, y}), [&](auto, auto op, auto op32, auto) -> lcs_status {
        for (int k = 0; k < std::max(reps, 1); ++k) {
            if (precision == LCS_PREC_FP64)
                hipLaunchKernelGGL((k_spmv<decltype(op)>), dim3(grid_for(op, kStreamGrid)),
                                   dim3(kBlock), 0, s, op, (const double *)x, (double *)y);
            else
                hipLaunchKernelGGL((k_spmv<decltype(op32)>),
                                   dim3(grid_for(op32, kStreamGrid)), dim3(kBlock), 0, s,
                                   op32, (const float *)x, (float *)y);
        }
        LAUNCH_CHECK();
        return LCS_OK;
    });
}

lcs_status lcs_cast_coef(lcs_ctx *c, const lcs_matrix *A, float *coef32, void *stream) {
    if (!c) return fail(LCS_EINVAL, "ctx is NULL");
    LCS_TRY(check_matrix(A));
    if (A->kind == LCS_CSR)
        return fail(LCS_EINVAL, "the FP32 copy of a CSR matrix is made inside each call");
    LCS_TRY(check_ptr(coef32, "coef32"));
    const int64_t n = (int64_t)A->nx * A->ny * A->nz * n_arrays(A->kind);
    hipLaunchKernelGGL(k_cast, dim3(flat_grid(n)), dim3(kBlock), 0, (hipStream_t)stream, A->coef,
                       coef32, n);
    LAUNCH_CHECK();
    return LCS_OK;
}

lcs_status lcs_build_local_domain(lcs_ctx *c, const lcs_matrix *A, const double *b,
                                  const double *x0, int32_t mode, int32_t thresh_kind,
                                  double theta, int32_t e_max, int32_t *idx, uint8_t *mask,
                                  int64_t *K, lcs_stats *st, void *stream) {
    if (!c) return fail(LCS_EINVAL, "ctx is NULL");
    LCS_TRY(check_matrix(A));
    LCS_TRY(plan_call(c, A, nullptr, kWhatDomain));
    LCS_TRY(prepare_matrix(c, A, (hipStream_t)stream));
    LCS_TRY(check_ptr(b, "b"));
    LCS_TRY(check_ptr(x0, "x0"));
    LCS_TRY(check_ptr(idx, "idx"));
    LCS_TRY(check_ptr(K, "K"));
    LCS_TRY(check_mode(mode, thresh_kind, theta, e_max));
    hipStream_t s = (hipStream_t)stream;
    return with_ops(c, A, nullptr, vec_ok({b, x0}), [&](auto sop, auto op, auto, auto) -> lcs_status {
        LCS_TRY(build_domain(c, sop, op, b, x0, mode, thresh_kind, theta, e_max, -1.0, idx, K, s));
        if (mask) {
            uint8_t *stamp;
            LCS_TRY(get_buf(c, B_STAMP, tiling_for(sop.n).npad, &stamp));
            HIP_TRY(hipMemcpyAsync(mask, stamp, (size_t)sop.n, hipMemcpyDeviceToDevice, s));
            LCS_TRY(wait_for(c, s));
        }
        if (st) {
            init_stats(st);
            st->K = *K;
            st->e_rounds = c->hsc->ms.grown;
            st->tau = c->hsc->ms.tau;
        }
        return LCS_OK;
    });
}

lcs_status lcs_gather_restricted(lcs_ctx *c, const lcs_matrix *A, const int32_t *idx, int64_t K,
                                 int32_t *row_ptr, int32_t *col, double *val, int64_t *nnz,
                                 void *stream) {
    if (!c) return fail(LCS_EINVAL, "ctx is NULL");
    LCS_TRY(check_matrix(A));
    LCS_TRY(plan_call(c, A, nullptr, kWhatGather));
    LCS_TRY(prepare_matrix(c, A, (hipStream_t)stream));
    const int64_t n = (int64_t)A->nx * A->ny * A->nz;
    if (K < 0 || K > n) return fail(LCS_EINVAL, "K out of range");
    if (K > 0) {
        LCS_TRY(check_ptr(idx, "idx"));
        LCS_TRY(check_ptr(row_ptr, "row_ptr"));
        LCS_TRY(check_ptr(col, "col"));
        LCS_TRY(check_ptr(val, "val"));
    }
    LCS_TRY(check_ptr(nnz, "nnz"));
    hipStream_t s = (hipStream_t)stream;
    return with_ops(c, A, nullptr, false, [&](auto sop, auto, auto, auto wtag) -> lcs_status {
        constexpr int W = decltype(wtag)::value;
        int32_t *inv, *len, *blocksum;
        LCS_TRY(get_buf(c, B_INV, n, &inv));
        LCS_TRY(set_inv(c, idx, K, n, inv, s));
        if (K == 0) {
            *nnz = 0;
            HIP_TRY(hipMemsetAsync(row_ptr, 0, sizeof(int32_t), s));
            LCS_TRY(wait_for(c, s));
            return LCS_OK;
        }
        Restricted<W> R;
        LCS_TRY(gather<W>(c, sop, idx, K, inv, nullptr, false, false, &R, s));
        // ELL -> CSR: row lengths, exclusive scan, fill
        LCS_TRY(get_buf(c, B_ROWLEN, K, &len));
        LCS_TRY(get_buf(c, B_BLOCKOFF, 2 * kMaxGrid, &blocksum));
        const Tiling T = tiling_for(K);
        hipLaunchKernelGGL(k_ell_rowlen, dim3(flat_grid(K)), dim3(kBlock), 0, s, R.B64.col, K, W, len);
        hipLaunchKernelGGL(k_scan_reduce, dim3(T.grid), dim3(kBlock), 0, s, (const int32_t *)len, K,
                           T.tiles_per_block, blocksum);
        hipLaunchKernelGGL(k_scan_apply, dim3(T.grid), dim3(kBlock), 0, s, (const int32_t *)len, K,
                           T.tiles_per_block, (const int32_t *)blocksum, row_ptr, c->dsc);
        hipLaunchKernelGGL(k_ell_to_csr, dim3(flat_grid(K)), dim3(kBlock), 0, s, R.B64.col, R.B64.val,
                           K, W, (const int32_t *)row_ptr, col, val);
        LAUNCH_CHECK();
        LCS_TRY(read_scalars(c, s));
        *nnz = c->hsc->gather_nnz;
        return LCS_OK;
    });
}

lcs_status lcs_gs_sweeps(lcs_ctx *c, const lcs_matrix *A, const double *b, double *x,
                         int32_t n_sweeps, void *stream) {
    if (!c) return fail(LCS_EINVAL, "ctx is NULL");
    LCS_TRY(check_matrix(A));
    LCS_TRY(plan_call(c, A, nullptr, kWhatPiece));
    LCS_TRY(prepare_matrix(c, A, (hipStream_t)stream));
    LCS_TRY(check_ptr(b, "b"));
    LCS_TRY(check_ptr(x, "x"));
    if (n_sweeps < 0) return fail(LCS_EINVAL, "n_sweeps < 0");
    hipStream_t s = (hipStream_t)stream;
    const int ncol = colours_of(A);
    if (ncol == 0) return fail(LCS_EINVAL, "Gauss-Seidel sweeps on a CSR matrix need its colouring");
    return with_ops(c, A, nullptr, vec_ok({b, x}), [&](auto, auto op, auto, auto) -> lcs_status {
        LCS_TRY(launch_sweeps(c, op, b, x, ncol, n_sweeps, s));
        LCS_TRY(wait_for(c, s));
        LCS_TRY(flush_prof(c));
        return LCS_OK;
    });
}

lcs_status lcs_solve_global(lcs_ctx *c, const lcs_matrix *A, const double *b, double *x,
                            const lcs_options *o, lcs_stats *st, void *stream) {
    if (!c) return fail(LCS_EINVAL, "ctx is NULL");
    LCS_TRY(check_matrix(A));
    LCS_TRY(check_options_for(o, A));
    LCS_TRY(plan_call(c, A, o, kWhatSolve));
    LCS_TRY(prepare_matrix(c, A, (hipStream_t)stream));
    LCS_TRY(check_ptr(b, "b"));
    LCS_TRY(check_ptr(x, "x"));
    lcs_stats local;
    if (!st) st = &local;
    init_stats(st);
    hipStream_t s = (hipStream_t)stream;
    Timers tm{c, s, true};
    const float *c32 = nullptr;
    LCS_TRY(tm.mark(0));
    LCS_TRY(ensure_coef32(c, A, o->precision == LCS_PREC_MIXED, &c32, s));
    const int64_t n = (int64_t)A->nx * A->ny * A->nz;
    return with_ops(c, A, c32, vec_ok({b, x}), [&](auto, auto op, auto op32, auto) -> lcs_status {
        LCS_TRY(launch_norm(c, b, n, &c->dsc->bnorm, s));
        LCS_TRY(tm.mark(3));
        SolveOut so;
        const lcs_status rs = solve_system(c, op, op32, colours_of(A), b, x, false,
                                           &c->dsc->bnorm, o->eps, o, s, &so, 0, uses_gmres(A));
        LCS_TRY(tm.mark(4));
        LCS_TRY(wait_for(c, s));
        LCS_TRY(flush_prof(c));
        const double bn = c->hsc->bnorm;
        st->its_global = so.its;
        st->n_outer = so.n_outer;
        st->relres_final = bn > 0 ? std::sqrt(so.rr) / bn : std::sqrt(so.rr);
        st->ms_global = tm.ms(0, 4);
        return rs;
    });
}

lcs_status lcs_solve_local(lcs_ctx *c, const lcs_matrix *A, const double *b, double *x,
                           const int32_t *idx, int64_t K, const lcs_options *o, lcs_stats *st,
                           void *stream) {
    if (!c) return fail(LCS_EINVAL, "ctx is NULL");
    LCS_TRY(check_matrix(A));
    LCS_TRY(check_options_for(o, A));
    LCS_TRY(plan_call(c, A, o, kWhatSolve));
    LCS_TRY(prepare_matrix(c, A, (hipStream_t)stream));
    LCS_TRY(check_ptr(b, "b"));
    LCS_TRY(check_ptr(x, "x"));
    const int64_t n = (int64_t)A->nx * A->ny * A->nz;
    if (K < 0 || K > n) return fail(LCS_EINVAL, "K out of range");
    if (K > 0) LCS_TRY(check_ptr(idx, "idx"));
    lcs_stats local;
    if (!st) st = &local;
    init_stats(st);
    st->K = K;
    hipStream_t s = (hipStream_t)stream;
    Timers tm{c, s, true};
    LCS_TRY(tm.mark(0));
    const float *c32 = nullptr;
    LCS_TRY(ensure_coef32(c, A, o->precision == LCS_PREC_MIXED, &c32, s));
    return with_ops(c, A, c32, vec_ok({b, x}), [&](auto sop, auto op, auto, auto wtag) -> lcs_status {
        constexpr int W = decltype(wtag)::value;
        LCS_TRY(launch_norm(c, b, n, &c->dsc->bnorm, s));
        int32_t *inv;
        LCS_TRY(get_buf(c, B_INV, n, &inv));
        LCS_TRY(set_inv(c, idx, K, n, inv, s));
        LCS_TRY(tm.mark(1));
        bool crit = false;
        LCS_TRY(local_phase<W>(c, A, sop, op, b, x, idx, K, inv, nullptr, o, st, tm, s, &crit));
        if (!crit)
            LCS_TRY(launch_resnorm(c, op, b, (const double *)x, (double *)nullptr,
                                   &c->dsc->bnorm, o->eps, s));
        LCS_TRY(read_scalars(c, s));
        LCS_TRY(flush_prof(c));
        LCS_TRY(finish_local(c, st));
        const double bn = c->hsc->bnorm;
        st->relres_after_local = bn > 0 ? std::sqrt(c->hsc->res.rr) / bn : std::sqrt(c->hsc->res.rr);
        st->relres_final = st->relres_after_local;
        st->ms_construct = tm.ms(0, 1);
        st->ms_local = tm.ms(1, 2);
        st->ms_smooth = tm.ms(2, 3);
        return LCS_OK;
    });
}

lcs_status lcs_solve_local_then_global(lcs_ctx *c, const lcs_matrix *A, const double *b,
                                       double *x, int32_t mode, int32_t thresh_kind,
                                       double theta, int32_t e_max, const lcs_options *o,
                                       lcs_stats *st, void *stream) {
    if (!c) return fail(LCS_EINVAL, "ctx is NULL");
    LCS_TRY(check_matrix(A));
    LCS_TRY(check_options_for(o, A));
    LCS_TRY(plan_call(c, A, o, kWhatSolve));
    LCS_TRY(prepare_matrix(c, A, (hipStream_t)stream));
    LCS_TRY(check_ptr(b, "b"));
    LCS_TRY(check_ptr(x, "x"));
    LCS_TRY(check_mode(mode, thresh_kind, theta, e_max));
    lcs_stats local;
    if (!st) st = &local;
    init_stats(st);
    hipStream_t s = (hipStream_t)stream;
    const int64_t n = (int64_t)A->nx * A->ny * A->nz;
    Timers tm{c, s, true};
    LCS_TRY(tm.mark(0));
    const float *c32 = nullptr;
    LCS_TRY(ensure_coef32(c, A, o->precision == LCS_PREC_MIXED, &c32, s));
    return with_ops(c, A, c32, vec_ok({b, x}), [&](auto sop, auto op, auto op32, auto wtag) -> lcs_status {
        constexpr int W = decltype(wtag)::value;
        int32_t *idx;
        LCS_TRY(get_buf(c, B_IDX, n, &idx));
        int64_t K = 0;
        // an odd number of one-pass sweeps starts from a copy of x that the
        // score pass writes (so that the last one writes x itself)
        double *xcopy = nullptr;
        if (one_pass_sweeps(op, colours_of(A), o->n_smooth, o->eps) && (o->n_smooth & 1))
            LCS_TRY(get_buf(c, B_GSX, (size_t)n, &xcopy));
        LCS_TRY(build_domain(c, sop, op, b, (const double *)x, mode, thresh_kind, theta, e_max,
                             o->eps, idx, &K, s, xcopy));
        st->K = K;
        st->e_rounds = c->hsc->ms.grown;
        st->tau = c->hsc->ms.tau;
        const double bn = c->hsc->bnorm;
        if (c->hsc->ms.conv0) {
            // x^(0) already meets the criterion: it is the solution, returned
            // as it is (no local solve, no smoothing), as the global PCG
            // returns an initial iterate that passes its first test
            const double rr0 = std::sqrt(c->hsc->ms.rr0);
            st->relres_after_local = st->relres_final = bn > 0 ? rr0 / bn : rr0;
            LCS_TRY(tm.mark(1));
            LCS_TRY(wait_for(c, s));
            LCS_TRY(flush_prof(c));
            st->ms_construct = tm.ms(0, 1);
            return LCS_OK;
        }
        LCS_TRY(tm.mark(1));
        double *score, *r0 = nullptr;
        int32_t *inv;
        LCS_TRY(get_buf(c, B_SCORE, n, &score));
        LCS_TRY(get_buf(c, B_INV, n, &inv));
        if (mode == LCS_MODE_RESIDUAL) r0 = score;
        // criterion after the local solve and smoothing (Algorithm 1 step
        // 8), formed in the last sweep pass where the sweep allows it
        bool crit = false;
        LCS_TRY(local_phase<W>(c, A, sop, op, b, x, idx, K, inv, r0, o, st, tm, s, &crit, xcopy));
        if (!crit)
            LCS_TRY(launch_resnorm(c, op, b, (const double *)x, (double *)nullptr,
                                   &c->dsc->bnorm, o->eps, s));
        // the end of the solve when the criterion holds (a global finish
        // records it again); the read's wait then covers every timer event
        LCS_TRY(tm.mark(4));
        LCS_TRY(read_scalars(c, s));
        LCS_TRY(finish_local(c, st));
        st->relres_after_local = bn > 0 ? std::sqrt(c->hsc->res.rr) / bn : std::sqrt(c->hsc->res.rr);
        lcs_status rs = LCS_OK;
        if (c->hsc->res.done) {
            st->relres_final = st->relres_after_local;
        } else {
            SolveOut so;
            rs = solve_system(c, op, op32, colours_of(A), b, x, false, &c->dsc->bnorm, o->eps,
                              o, s, &so, 0, uses_gmres(A));
            st->its_global = so.its;
            st->n_outer += so.n_outer;
            st->relres_final = bn > 0 ? std::sqrt(so.rr) / bn : std::sqrt(so.rr);
            LCS_TRY(tm.mark(4));
            LCS_TRY(wait_for(c, s));
        }
        LCS_TRY(flush_prof(c));
        st->ms_construct = tm.ms(0, 1);
        st->ms_local = tm.ms(1, 2);
        st->ms_smooth = tm.ms(2, 3);
        st->ms_global = tm.ms(3, 4);
        return rs;
    });
}

lcs_status lcs_solve_global_batched(lcs_ctx *c, const lcs_matrix *A, int32_t G, const double *b,
                                    double *x, const lcs_options *o, lcs_stats *st, void *stream) {
    return solve_batched(c, A, G, b, x, 0, 0, 0, 0.0, 0, o, st, stream);
}

lcs_status lcs_solve_local_then_global_batched(lcs_ctx *c, const lcs_matrix *A, int32_t G,
                                               const double *b, double *x, int32_t mode,
                                               int32_t thresh_kind, double theta, int32_t e_max,
                                               const lcs_options *o, lcs_stats *st, void *stream) {
    return solve_batched(c, A, G, b, x, 1, mode, thresh_kind, theta, e_max, o, st, stream);
}

lcs_status lcs_set_kernel_timing(lcs_ctx *c, int32_t what) {
    if (!c) return fail(LCS_EINVAL, "ctx is NULL");
    if (what < LCS_TIME_NONE || what > LCS_TIME_SCORE) return fail(LCS_EINVAL, "timing class");
    c->prof_what = what;
    c->prof_used = 0;
    c->prof_ms = 0.0;
    c->prof_launches = 0;
    return LCS_OK;
}

lcs_status lcs_set_colour_blocking(lcs_ctx *c, int32_t on) {
    if (!c) return fail(LCS_EINVAL, "ctx is NULL");
    c->colour_blocks = on != 0;
    return LCS_OK;
}

lcs_status lcs_set_short_columns(lcs_ctx *c, int32_t on) {
    if (!c) return fail(LCS_EINVAL, "ctx is NULL");
    c->short_cols = on != 0;
    return LCS_OK;
}

lcs_status lcs_set_tiling(lcs_ctx *c, int32_t march_rows, int32_t nontemporal) {
    if (!c) return fail(LCS_EINVAL, "ctx is NULL");
    if (nontemporal > 1) return fail(LCS_EINVAL, "nontemporal must be -1, 0 or 1");
    c->march_rows = march_rows < 0 ? -1 : march_rows;
    c->nontemporal = nontemporal < 0 ? -1 : nontemporal;
    return LCS_OK;
}

lcs_status lcs_get_kernel_timing(lcs_ctx *c, double *ms_total, int64_t *launches) {
    if (!c || !ms_total || !launches) return fail(LCS_EINVAL, "NULL argument");
    *ms_total = c->prof_ms;
    *launches = c->prof_launches;
    return LCS_OK;
}

lcs_status lcs_assemble_heat(lcs_ctx *c, int32_t nx, int32_t ny, double inv_dt, double power,
                             double t_left, double t_right, const double *t_lin,
                             const double *t_old, double *coef, double *b, void *stream) {
    if (!c) return fail(LCS_EINVAL, "ctx is NULL");
    if (nx < 1 || ny < 1) return fail(LCS_EINVAL, "grid sizes");
    if (!(t_left > 0.0) || !(t_right > 0.0)) return fail(LCS_EINVAL, "boundary temperatures must be > 0");
    LCS_TRY(check_ptr(t_lin, "t_lin"));
    LCS_TRY(check_ptr(t_old, "t_old"));
    LCS_TRY(check_ptr(coef, "coef"));
    LCS_TRY(check_ptr(b, "b"));
    const int64_t n = (int64_t)nx * ny;
    hipLaunchKernelGGL(k_assemble_heat, dim3(flat_grid(n)), dim3(kBlock), 0, (hipStream_t)stream,
                       nx, ny, inv_dt, power, t_left, t_right, t_lin, t_old, coef, b);
    LAUNCH_CHECK();
    return LCS_OK;
}

lcs_status lcs_norm2_diff(lcs_ctx *c, const double *a, const double *b, int64_t n, double *out,
                          void *stream) {
    if (!c) return fail(LCS_EINVAL, "ctx is NULL");
    if (n < 0) return fail(LCS_EINVAL, "n < 0");
    LCS_TRY(check_ptr(out, "out"));
    if (n == 0) {
        *out = 0.0;
        return LCS_OK;
    }
    LCS_TRY(check_ptr(a, "a"));
    LCS_TRY(check_ptr(b, "b"));
    hipStream_t s = (hipStream_t)stream;
    const Launch L = dims_for(n);
    hipLaunchKernelGGL(k_norm2_diff, dim3(L.grid), dim3(kBlock), 0, s, a, b, n, L.chunk,
                       slot(c, kPtNorm));
    hipLaunchKernelGGL(k_fin_norm, dim3(1), dim3(kBlock), 0, s, (const double *)slot(c, kPtNorm),
                       L.grid, &c->dsc->scratch_norm);
    LAUNCH_CHECK();
    LCS_TRY(read_scalars(c, s));
    *out = c->hsc->scratch_norm;
    return LCS_OK;
}

lcs_status lcs_assemble_logk(lcs_ctx *c, int32_t kind, int32_t nx, int32_t ny, int32_t nz,
                             double inv_dt, const double *logk, double *coef, void *stream) {
    if (!c) return fail(LCS_EINVAL, "ctx is NULL");
    if (kind != LCS_STENCIL5_2D && kind != LCS_STENCIL7_3D)
        return fail(LCS_EINVAL, "log-conductivity assembly exists for the 5- and 7-point operators");
    if (nx < 1 || ny < 1 || nz < 1 || (kind == LCS_STENCIL5_2D && nz != 1))
        return fail(LCS_EINVAL, "grid sizes");
    LCS_TRY(check_ptr(logk, "logk"));
    LCS_TRY(check_ptr(coef, "coef"));
    const int64_t n = (int64_t)nx * ny * nz;
    hipStream_t s = (hipStream_t)stream;
    if (kind == LCS_STENCIL5_2D)
        hipLaunchKernelGGL(k_assemble_logk<2>, dim3(flat_grid(n)), dim3(kBlock), 0, s, nx, ny, nz,
                           inv_dt, logk, coef);
    else
        hipLaunchKernelGGL(k_assemble_logk<3>, dim3(flat_grid(n)), dim3(kBlock), 0, s, nx, ny, nz,
                           inv_dt, logk, coef);
    LAUNCH_CHECK();
    return LCS_OK;
}

lcs_status lcs_grad_logk(lcs_ctx *c, int32_t kind, int32_t nx, int32_t ny, int32_t nz,
                         const double *logk, const double *x, const double *lam, double *grad,
                         void *stream) {
    if (!c) return fail(LCS_EINVAL, "ctx is NULL");
    if (kind != LCS_STENCIL5_2D && kind != LCS_STENCIL7_3D)
        return fail(LCS_EINVAL, "log-conductivity gradient exists for the 5- and 7-point operators");
    if (nx < 1 || ny < 1 || nz < 1 || (kind == LCS_STENCIL5_2D && nz != 1))
        return fail(LCS_EINVAL, "grid sizes");
    LCS_TRY(check_ptr(logk, "logk"));
    LCS_TRY(check_ptr(x, "x"));
    LCS_TRY(check_ptr(lam, "lam"));
    LCS_TRY(check_ptr(grad, "grad"));
    const int64_t n = (int64_t)nx * ny * nz;
    hipStream_t s = (hipStream_t)stream;
    if (kind == LCS_STENCIL5_2D)
        hipLaunchKernelGGL(k_grad_logk<2>, dim3(flat_grid(n)), dim3(kBlock), 0, s, nx, ny, nz, logk,
                           x, lam, grad);
    else
        hipLaunchKernelGGL(k_grad_logk<3>, dim3(flat_grid(n)), dim3(kBlock), 0, s, nx, ny, nz, logk,
                           x, lam, grad);
    LAUNCH_CHECK();
    return LCS_OK;
}

lcs_status lcs_build_local_domain_static(const lcs_matrix *A, const double *b, const double *x0,
                                         int32_t mode, int32_t thresh_kind, double theta,
                                         int32_t e_max, int32_t *idx, uint8_t *mask, int64_t *K,
                                         lcs_stats *st, void *stream) {
    LCS_TRY(check_matrix(A));
    if (A->kind == LCS_CSR)
        return fail(LCS_EINVAL, "the allocation-free local domain takes the stencil kinds");
    const int64_t n = (int64_t)A->nx * A->ny * A->nz;
    if (n > kStaticMaxN)
        return fail(LCS_EINVAL, "the allocation-free local domain takes at most 2^21 cells, got " +
                                    std::to_string(n));
    LCS_TRY(check_ptr(b, "b"));
    LCS_TRY(check_ptr(x0, "x0"));
    LCS_TRY(check_ptr(idx, "idx"));
    LCS_TRY(check_ptr(K, "K"));
    LCS_TRY(check_mode(mode, thresh_kind, theta, e_max));
    void *p = nullptr;
    int dev = 0;
    LCS_TRY(static_scratch(&p, &dev));
    // a context on the stack whose state, partials and buffers lie in the
    // scratch array; scalars come back into pageable host memory
    lcs_ctx t;
    t.device = dev;
    t.ws = static_cast<char *>(p);
    t.ws_bytes = kStaticScratchBytes;
    t.dsc = reinterpret_cast<Scalars *>(t.ws);
    t.partials = reinterpret_cast<double *>(t.ws + align_up(sizeof(Scalars)));
    Scalars host_state;
    t.hsc = &host_state;
    LCS_TRY(plan_call(&t, A, nullptr, kWhatDomain));
    hipStream_t s = (hipStream_t)stream;
    return with_ops(&t, A, nullptr, vec_ok({b, x0}), [&](auto sop, auto op, auto, auto) -> lcs_status {
        LCS_TRY(build_domain(&t, sop, op, b, x0, mode, thresh_kind, theta, e_max, -1.0, idx, K, s));
        if (mask) {
            uint8_t *stamp;
            LCS_TRY(get_buf(&t, B_STAMP, tiling_for(sop.n).npad, &stamp));
            HIP_TRY(hipMemcpyAsync(mask, stamp, (size_t)sop.n, hipMemcpyDeviceToDevice, s));
            HIP_TRY(hipStreamSynchronize(s));
        }
        if (st) {
            init_stats(st);
            st->K = *K;
            st->e_rounds = host_state.ms.grown;
            st->tau = host_state.ms.tau;
        }
        return LCS_OK;
    });
}

}  // extern "C"
