// internal.h -- shared declarations of the apcg runtime (host side) and the
// device helpers every kernel file uses.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <cstdint>
#include <functional>
#include <memory>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "../../include/apcg.h"

namespace apcg {

// ---------------------------------------------------------------------------
// errors and counters
// ---------------------------------------------------------------------------
apcg_status set_error(apcg_status code, const std::string &msg);
apcg_status hip_error(hipError_t e, const char *what);

struct Counters {
    std::atomic<int64_t> kernel_launches{0}, graph_launches{0}, host_syncs{0}, host_polls{0},
        d2h_copies{0}, h2d_copies{0}, stream_waits{0};
};
extern Counters g_counters;

#define APCG_HIP(call)                                                   \
    do {                                                                 \
        hipError_t e__ = (call);                                         \
        if (e__ != hipSuccess) return ::apcg::hip_error(e__, #call);     \
    } while (0)

#define APCG_CHECK_LAUNCH(what)                                          \
    do {                                                                 \
        ::apcg::g_counters.kernel_launches++;                            \
        hipError_t e__ = hipGetLastError();                              \
        if (e__ != hipSuccess) return ::apcg::hip_error(e__, what);      \
    } while (0)

// ---------------------------------------------------------------------------
// pooled events and the access registry (ordering rule of Section 3.1.2)
// ---------------------------------------------------------------------------
struct Event {
    hipEvent_t e = nullptr;
    int device = 0;
    ~Event();
};
using EventRef = std::shared_ptr<Event>;
EventRef event_get(int device);  // un-recorded event from the device's pool

struct Record {
    uint64_t writer_ctx = 0;  // 0: never written through the library
    EventRef write_ev;
    std::vector<std::pair<uint64_t, EventRef>> readers;  // reads since the last write
};

enum AccessMode { ACC_R = 1, ACC_W = 2, ACC_RW = 3 };
struct Acc {
    Record *rec;
    int mode;
};

extern std::recursive_mutex g_mu;  // guards every Record and the deferred list

// Deferred release: fn runs once every event in deps has completed.
void defer_release(std::vector<EventRef> deps, std::function<void()> fn);
void reap();                       // runs the releases whose events completed
std::vector<EventRef> record_deps(const Record &r);

// ---------------------------------------------------------------------------
// solve workspace and per-context scratch
// ---------------------------------------------------------------------------
struct SolveState;  // device struct, defined in pcg.hip

// Everything a captured PCG graph bakes into its kernel arguments: a cached
// graph is replayed only for an identical key.
struct GraphKey {
    uint64_t mat_uid;
    const void *rowptr, *col, *val, *x, *ws, *state, *partials, *prod;
    int64_t ws_cap, pb_vec, lds_bytes;
    int32_t n, K, tb, g_prod, rpb, g_vec, lds_nnz, pc, norm;
    bool operator==(const GraphKey &o) const {
        return mat_uid == o.mat_uid && rowptr == o.rowptr && col == o.col && val == o.val && x == o.x &&
               ws == o.ws && state == o.state && partials == o.partials && prod == o.prod && ws_cap == o.ws_cap &&
               pb_vec == o.pb_vec && lds_bytes == o.lds_bytes && n == o.n && K == o.K && tb == o.tb &&
               g_prod == o.g_prod && rpb == o.rpb && g_vec == o.g_vec && lds_nnz == o.lds_nnz && pc == o.pc &&
               norm == o.norm;
    }
};

struct GraphEntry {
    GraphKey key;
    hipGraphExec_t exec = nullptr;
    hipGraph_t graph = nullptr;
};

constexpr int kMaxBlocks = 8192;    // reduction partials per kernel
constexpr int kPartialSlots = 8;    // kMaxBlocks-sized slices of the partials buffer
constexpr int kMaxLookahead = 8;
// Largest staged chunk (nonzeros): 12 bytes each must fit the 64 KiB of LDS
// one workgroup may take.
constexpr int kStreamMaxNnz = 5376;
inline bool stream_fits(const apcg_mat_s *A, int tb);


struct Workspace {
    int64_t cap = 0;          // elements per vector
    double *base = nullptr;   // 6 * cap doubles: r, dinv, p0, p1, w, z
    SolveState *state = nullptr;  // 256 bytes
    double *r() const { return base; }
    double *dinv() const { return base + cap; }
    double *p(int i) const { return base + (2 + i) * cap; }
    double *w() const { return base + 4 * cap; }
    double *z() const { return base + 5 * cap; }  // D^-1 r, stored by the update for the product's gather
};

}  // namespace apcg

// ---------------------------------------------------------------------------
// opaque handle structs
// ---------------------------------------------------------------------------
struct apcg_ctx_s {
    uint64_t id = 0;
    int32_t device = 0;
    int32_t type = APCG_STREAM_DEFAULT;
    hipStream_t stream = nullptr;
    bool is_default_global = false;
    double *partials = nullptr;      // kPartialSlots * kMaxBlocks
    int32_t *pinned_flags = nullptr; // kMaxLookahead host-pinned words
    apcg::EventRef poll_ev[apcg::kMaxLookahead];
    apcg::Workspace ws;
    std::vector<apcg::GraphEntry> graphs;
    // kernel timing (solve with kernel_timing = 1)
    std::vector<hipEvent_t> tev;     // pairs per timed launch
    std::vector<int> tkind;          // kind of each pair
    int32_t tpairs = 0;
    apcg::EventRef tdone;
};

struct apcg_scalar_s {
    int32_t device = 0;
    double *d = nullptr;  // slot in the device scalar pool
    int64_t slot = -1;
    apcg::Record rec;
    uint64_t mark_id = 0;  // id for dependency marking, assigned on request
};

struct apcg_vec_s {
    int32_t device = 0;
    double *d = nullptr;
    int64_t n = 0;
    apcg::Record rec;
    uint64_t mark_id = 0;
};

struct apcg_mat_s {
    uint64_t uid = 0;  // never reused: cached graphs are keyed on it, not on the handle's address
    int32_t device = 0;
    int32_t n = 0;
    int64_t nnz = 0;
    const int32_t *rowptr = nullptr, *col = nullptr;
    const double *val = nullptr;
    apcg_spmv_config cfg{};
    int64_t max_block_nnz[2] = {0, 0};  // most nonzeros in any 256- / 512-row block
    // Sliced layout (64-row slices, entries of a slice column-major), used
    // by the SELL schedule: built on the host at wrap time (slice offset and
    // width), filled on the device from the CSR arrays at the start of every
    // solve that uses it.
    std::vector<int32_t> sell_meta_h;  // [2 * nslices]: offset, width
    int64_t sell_entries = 0;          // -1: too large for int32 offsets
    int32_t sell_maxw = 0;
    int32_t *sell_meta = nullptr;      // device copies, allocated on first use
    int32_t *sell_col = nullptr;
    double *sell_val = nullptr;
    // Sliced-diagonal layout (SDIA schedule): the rows of a 64-row slice
    // share one sorted list of column offsets (column - row); per offset a
    // 64-bit mask says which rows hold that entry, and the values are stored
    // column-major by offset.  The offsets and masks are built on the host
    // the first time the schedule is selected (a snapshot of the sparsity
    // pattern), the values are refilled from the CSR arrays at the start of
    // every solve that uses it.
    int32_t sdia_state = 0;          // 0: not analysed, 1: available, -1: not applicable
    const char *sdia_reason = "";    // why not applicable
    int32_t sdia_u = 0;              // value slots per slice (largest offset count of any slice)
    int32_t sdia_mp = 0;             // offset / mask slots per slice: 8, 16 or 32 (>= sdia_u)
    int32_t sdia_ps = 0;             // plane stride in slices for plane marching (0: none)
    int32_t sdia_sym = 0;            // 1: the pattern is structurally symmetric
    int32_t *sdia_off = nullptr;     // device [nslices * sdia_mp] offsets (padding 0), then
                                     //   [nslices * sdia_mp] partner slots of the entries left of
                                     //   the diagonal, then the value-symmetry flag (64 ints; set
                                     //   by the analysis, only ever cleared on the device)
    uint64_t *sdia_msk = nullptr;    // device [nslices * sdia_mp] row masks, padding 0
    double *sdia_val = nullptr;      // device [nslices * sdia_u * 64] values, absent entries 0
    // Diagonal layout (DIA schedule): the whole matrix has at most
    // kDiaMaxDiags distinct column offsets; diagonal k is an array of
    // n rounded up to 64 values (value of row i at offset dia_off[k], 0 where
    // the row has no such entry).  The offsets are found on the host the
    // first time the schedule is selected; the values are refilled from the
    // CSR arrays at the start of every solve that uses it.
    int32_t dia_state = 0;           // 0: not analysed, 1: available, -1: not applicable
    const char *dia_reason = "";
    int32_t dia_nd = 0;              // distinct offsets (diagonals)
    int32_t dia_ndt = 0;             // diagonals the kernel walks (5, 7 or 9 >= dia_nd; the rest all zero)
    int32_t dia_sym = 0;             // 1: the offset set is symmetric (o present <=> -o present)
    int32_t dia_ps = 0;              // plane stride in 64-row slices (offset +-64 dia_ps present), 0: none
    int32_t dia_off_h[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    int32_t *dia_tab = nullptr;      // device int32[32]: offsets [0..8], partner diagonal of each
                                     //   negative offset [9..17] (-1: none), value-symmetry flag [18]
                                     //   (set by the analysis when dia_sym, only ever cleared on the device)
    double *dia_val = nullptr;       // device [dia_ndt][n rounded up to 64]
    apcg::Record rec;
    uint64_t mark_id = 0;
    std::string tune_class;  // pattern class of the tuning key (tune.hip), computed once
};

struct apcg_info_s {
    int32_t device = 0;
    int32_t count = 0;
    apcg_solve_info *d = nullptr;
    apcg::Record rec;
};

struct apcg_timer_s {
    apcg::EventRef start, stop;
};

namespace apcg {

// context helpers (runtime.hip)
apcg_status resolve_ctx(apcg_ctx in, int device, apcg_ctx *out);  // NULL -> global default
apcg_status op_begin(apcg_ctx c, const Acc *acc, int n);
apcg_status op_end(apcg_ctx c, const Acc *acc, int n);
apcg_status ensure_workspace(apcg_ctx c, int64_t n);
// Whether two vectors share memory: the same handle, or address ranges
// [d, d + n) that overlap (an empty range overlaps nothing).
inline bool vec_overlap(const apcg_vec_s *a, const apcg_vec_s *b) {
    const uintptr_t a0 = (uintptr_t)a->d, a1 = (uintptr_t)(a->d + a->n);
    const uintptr_t b0 = (uintptr_t)b->d, b1 = (uintptr_t)(b->d + b->n);
    return a == b || (a->n > 0 && b->n > 0 && a0 < b1 && b0 < a1);
}
// rows per tile of the segmented batched schedules (apcg_solve_opts.batch_tile_rows)
constexpr int32_t kDefaultBatchTileRows = 1024;
inline bool valid_batch_tile_rows(int32_t tr) { return tr == 0 || (tr >= 256 && tr <= 8192 && tr % 256 == 0); }
inline int32_t batch_tile_rows(const apcg_solve_opts &o) {
    return o.batch_tile_rows > 0 ? o.batch_tile_rows : kDefaultBatchTileRows;
}
// rows per tile once few rows still run (apcg_solve_opts.batch_tail_tile_rows):
// 0 when the tiles are kept
constexpr int32_t kDefaultBatchTailRows = 256;
inline bool valid_batch_tail_rows(int32_t tr) { return tr == -1 || valid_batch_tile_rows(tr); }
inline int32_t batch_tail_rows(const apcg_solve_opts &o) {
    const int32_t t = o.batch_tail_tile_rows > 0 ? o.batch_tail_tile_rows
                      : o.batch_tail_tile_rows == 0 ? kDefaultBatchTailRows : 0;
    return t < batch_tile_rows(o) ? t : 0;
}
// tuning table (tune.hip): the key of a pattern, lookups and inserts
std::string pattern_class(int64_t n, int64_t nnz, const int32_t *rp, const int32_t *cl);
std::string tune_key(const std::string &arch, const std::string &cls, int64_t n, int64_t nnz);
apcg_status device_arch(int device, std::string *out);
apcg_status mat_tune_key(apcg_mat_s *A, std::string *key);
bool tune_lookup(const std::string &key, int32_t v[4], double *us);
void tune_insert(const std::string &key, const int32_t v[4], double us);
// diagonal (DIA) layout (pcg.hip)
constexpr int kDiaMaxDiags = 9;
apcg_status dia_analyse(apcg_mat_s *A);
apcg_status prepare_dia(apcg_mat_s *A, hipStream_t s);
// one-workgroup persistent Jacobi-PCG (persist.hip): p is n doubles of device
// memory the workgroup shares; maxrow the longest row (< 0: unknown)
int persistent_rows_per_thread(int64_t n);
apcg_status launch_pcg_wg(hipStream_t st, int32_t n, const int32_t *rowptr, const int32_t *col, const double *val,
                          const double *b, double *x, double *p, double rtol, int32_t maxit, int x0_zero, int pc,
                          int norm_pre, int32_t maxrow, apcg_solve_info *out);
void batch_cache_release(uint64_t ctx_id, int device);  // batched.hip
// sliced-diagonal pattern analysis (pcg.hip): synchronous, once per matrix
apcg_status sdia_analyse(apcg_mat_s *A);
// queues the refill of the sliced-diagonal values on stream s (pcg.hip);
// analyses first if needed, APCG_ERR_UNSUPPORTED when the layout does not apply
apcg_status prepare_sdia(apcg_mat_s *A, hipStream_t s);
// Row-helper width for an analysed sliced-diagonal matrix: 5 or 7 when the
// 8-wide copy holds at most that many offsets per slice, else its width.
inline int sdia_walk(const apcg_mat_s *A) {
    if (A->sdia_mp != 8) return A->sdia_mp;
    return A->sdia_u <= 5 ? 5 : A->sdia_u <= 7 ? 7 : 8;
}
// Jacobi-PCG solve with registry marking (pcg.hip); hist (2 hist_cap doubles,
// device) receives alpha_k and beta_k of the first hist_cap iterations.
// gate (device int32[2], may be null): read by the solve's first kernels --
// gate[0] == 0 turns the whole solve into no-ops (x untouched, record of 0
// iterations), otherwise gate[1] replaces maxit on the device (the host
// queues at most maxit iterations).
apcg_status pcg_solve_marked(apcg_ctx ctx, apcg_mat A, apcg_vec b, apcg_vec x, double rtol, int32_t maxit,
                             const apcg_solve_opts *opts, apcg_info info, int32_t info_index, double *hist,
                             int32_t hist_cap, const int32_t *gate = nullptr);
void seg_cache_release(uint64_t ctx_id, int device);    // batched.hip
void learn_cache_release(uint64_t ctx_id, int device);  // learn.hip
void fcg_cache_release(uint64_t ctx_id, int device);    // fcg.hip
void bfcg_cache_release(uint64_t ctx_id, int device);   // batched_fcg.hip
void tq_cache_release(uint64_t ctx_id, int device);     // tfqmr.hip
// dependency-marking ids of library objects (intent.hip): an object's id
// maps to its Record until the object is destroyed
uint64_t intent_object_id(uint64_t *slot, int device, Record *rec);
void intent_forget(uint64_t id);
// Standardises X[B][16] in place with mean/std and writes the network's
// coefficients C[B][9] (learn.hip); ordered on ctx's stream.
apcg_status mlp_infer(apcg_ctx ctx, const float *params, const float *mean, const float *std, float *X, int32_t B,
                      float *C);
void spmv_default_config(int32_t n, int64_t nnz, apcg_spmv_config *cfg);
int32_t normalise_blocks(int32_t blocks, int64_t units);  // multiple of 8, <= kMaxBlocks

// kernel launchers (blas.hip)
apcg_status launch_dot(hipStream_t s, const double *x, const double *y, int64_t n, double *out, int take_sqrt,
                       double *partials);
apcg_status launch_axpy(hipStream_t s, double *y, const double *a, double sign, const double *x, int64_t n);
apcg_status launch_aypx(hipStream_t s, double *y, const double *b, const double *x, int64_t n);
apcg_status launch_scale(hipStream_t s, double *x, const double *a, int64_t n);
apcg_status launch_copy(hipStream_t s, double *dst, const double *src, int64_t n);
apcg_status launch_fill(hipStream_t s, double *x, double v, int64_t n);
apcg_status launch_scalar_op(hipStream_t s, int op, double *out, const double *a, const double *b);
apcg_status launch_scalar_set(hipStream_t s, double *out, double v);
apcg_status launch_spmv(hipStream_t s, const apcg_mat_s *A, const double *x, double *y);

inline bool stream_fits(const apcg_mat_s *A, int tb) {
    return (tb == 256 || tb == 512) && A->max_block_nnz[tb == 512 ? 1 : 0] <= kStreamMaxNnz;
}

// Grid and chunk for an elementwise pass over n entries: 2048 workgroups at
// most, chunks a multiple of 64 entries (512-byte aligned for doubles).
inline void elementwise_grid(int64_t n, int *G, int64_t *per_block) {
    int64_t units = (n + 63) / 64;
    *G = normalise_blocks(2048, units);
    int64_t pb = (n + *G - 1) / *G;
    *per_block = ((pb + 63) / 64) * 64;
    if (*per_block < 64) *per_block = 64;
}

}  // namespace apcg

// ---------------------------------------------------------------------------
// device helpers
// ---------------------------------------------------------------------------
namespace apcg {
namespace dev {

// Workgroups are dealt round-robin to the 8 XCDs (block b runs on XCD b % 8).
// Renumber them so XCD x owns the contiguous logical range
// [x * G/8, (x+1) * G/8); G is always a multiple of 8.
__device__ __forceinline__ int xcd_block(int b, int G) { return (b & 7) * (G >> 3) + (b >> 3); }

struct Chunk {
    int64_t lo, hi;
};

// The contiguous range [lo, hi) of the logical workgroup, clipped to n.
__device__ __forceinline__ Chunk block_chunk(int64_t n, int64_t per_block) {
    const int lb = xcd_block(blockIdx.x, gridDim.x);
    int64_t lo = (int64_t)lb * per_block;
    int64_t hi = lo + per_block;
    if (hi > n) hi = n;
    return {lo, hi};
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Sum of v over the block; the result is valid in thread 0.
template <int BS, int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV], double *lds) {
    constexpr int NW = BS / 64;
#pragma unroll
    for (int k = 0; k < NV; ++k) v[k] = wave_sum(v[k]);
    const int wid = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (lane == 0) {
#pragma unroll
        for (int k = 0; k < NV; ++k) lds[k * NW + wid] = v[k];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < NV; ++k) {
            double s = lds[k * NW];
            for (int w = 1; w < NW; ++w) s += lds[k * NW + w];
            v[k] = s;
        }
    }
}

// First stage of a deterministic reduction: the block's sums go to
// partials[k*G + slot].  No fence and no atomic: the consumer is a later
// kernel, and the kernel boundary makes the partials visible to it.
template <int BS, int NV>
__device__ __forceinline__ void store_partials(double (&v)[NV], double *partials, int G, int slot) {
    __shared__ double lds[NV * (BS / 64)];
    block_sum<BS, NV>(v, lds);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < NV; ++k) partials[k * G + slot] = v[k];
    }
}

// Second stage, run redundantly by every workgroup of the consuming kernel:
// thread t adds partials[k*G + i] for i = t, t + BS, ... in index order, then
// the fixed block tree.  Every workgroup of one kernel runs the same
// instruction sequence, so all of them obtain bit-identical totals.  All
// threads of the block return the totals.
template <int BS, int NV>
__device__ __forceinline__ void reduce_partials(const double *partials, int G, double (&out)[NV]) {
    __shared__ double lds[NV * (BS / 64)];
    __shared__ double bcast[NV];
    double t[NV];
#pragma unroll
    for (int k = 0; k < NV; ++k) t[k] = 0.0;
    // four of a thread's partials loaded before they are added (the same
    // order of addition): the prologue's latency is that of one load
    constexpr int UA = 4;
    int i = threadIdx.x;
    for (; i + (UA - 1) * BS < G; i += UA * BS) {
        double u[UA][NV];
#pragma unroll
        for (int a = 0; a < UA; ++a)
#pragma unroll
            for (int k = 0; k < NV; ++k) u[a][k] = partials[k * G + i + a * BS];
#pragma unroll
        for (int a = 0; a < UA; ++a)
#pragma unroll
            for (int k = 0; k < NV; ++k) t[k] += u[a][k];
    }
    for (; i < G; i += BS) {
#pragma unroll
        for (int k = 0; k < NV; ++k) t[k] += partials[k * G + i];
    }
    block_sum<BS, NV>(t, lds);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < NV; ++k) bcast[k] = t[k];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < NV; ++k) out[k] = bcast[k];
}


// ---------------------------------------------------------------------------
// learned-preconditioner features (learn.hip, batched_fcg.hip)
// ---------------------------------------------------------------------------
// Per-row statistics, accumulated over rows: min(1 - R_i), max(1 + R_i) with
// R_i = sum |offdiag| / |d_i| (Gershgorin bounds of D^-1 A), min / max / sum
// of ln d_i, sum over rows with off-diagonals of ln(max |off| / min |off|)
// and the count of such rows.
struct RowStats {
    double v[7] = {INFINITY, -INFINITY, INFINITY, -INFINITY, 0.0, 0.0, 0.0};
};

__device__ inline void row_stats_add(RowStats &a, const int32_t *__restrict__ rowptr, const int32_t *__restrict__ col,
                                     const double *__restrict__ val, int64_t i) {
    double d = 0.0, off = 0.0, omax = 0.0, omin = INFINITY;
    for (int k = rowptr[i]; k < rowptr[i + 1]; ++k) {
        const double x = val[k];
        if (col[k] == (int)i) d = x;
        else {
            const double ax = fabs(x);
            off += ax;
            omax = fmax(omax, ax);
            omin = fmin(omin, ax);
        }
    }
    const double R = off / fabs(d), ld = log(d);
    a.v[0] = fmin(a.v[0], 1.0 - R);
    a.v[1] = fmax(a.v[1], 1.0 + R);
    a.v[2] = fmin(a.v[2], ld);
    a.v[3] = fmax(a.v[3], ld);
    a.v[4] += ld;
    if (omax > 0.0) {
        a.v[5] += log(omax / omin);
        a.v[6] += 1.0;
    }
}

__device__ inline void row_stats_merge(RowStats &a, const double *b) {
    a.v[0] = fmin(a.v[0], b[0]);
    a.v[1] = fmax(a.v[1], b[1]);
    a.v[2] = fmin(a.v[2], b[2]);
    a.v[3] = fmax(a.v[3], b[3]);
    a.v[4] += b[4];
    a.v[5] += b[5];
    a.v[6] += b[6];
}

// Merges the RowStats of a workgroup's BS threads by a fixed tree in LDS
// (sh: 7 x BS doubles); the result is valid in thread 0.
template <int BS>
__device__ inline void row_stats_block(RowStats &a, double (*sh)[BS]) {
    for (int k = 0; k < 7; ++k) sh[k][threadIdx.x] = a.v[k];
    __syncthreads();
    for (int off = BS / 2; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) {
            RowStats t;
            double b[7];
            for (int k = 0; k < 7; ++k) {
                t.v[k] = sh[k][threadIdx.x];
                b[k] = sh[k][threadIdx.x + off];
            }
            row_stats_merge(t, b);
            for (int k = 0; k < 7; ++k) sh[k][threadIdx.x] = t.v[k];
        }
        __syncthreads();
    }
    for (int k = 0; k < 7; ++k) a.v[k] = sh[k][0];
}

__device__ inline double row_logdiag(const int32_t *__restrict__ rowptr, const int32_t *__restrict__ col,
                                     const double *__restrict__ val, int64_t i) {
    double d = 0.0;
    for (int k = rowptr[i]; k < rowptr[i + 1]; ++k)
        if (col[k] == (int)i) d = val[k];
    return log(d);
}

// Eigenvalues below x of the symmetric tridiagonal with diagonal
// 1/al_j + be_{j-1}/al_{j-1} and squared off-diagonal be_j / al_j^2 (the
// CG-Lanczos tridiagonal of alpha_j = al[j], beta_j = be[j]): negative
// pivots of the LDL' factorisation of T - x I (Sturm sequence; Golub & Van
// Loan, Sec. 8.4.1), a zero pivot replaced by a tiny negative one.
__device__ inline int sturm_below(const double *al, const double *be, int m, double x) {
    int cnt = 0;
    double q = 1.0;
    for (int j = 0; j < m; ++j) {
        double d = 1.0 / al[j] - x;
        if (j > 0) d += be[j - 1] / al[j - 1] - (be[j - 1] / (al[j - 1] * al[j - 1])) / q;
        q = d;
        if (fabs(q) < 1e-300) q = -1e-300;
        if (q < 0.0) ++cnt;
    }
    return cnt;
}

// Ritz values of at most 16 CG steps, one workgroup: threads j < m write the
// CG-Lanczos tridiagonal (diagonal d, squared off-diagonal e2) to LDS, then
// thread i < m bisects for the i-th smallest eigenvalue on the Sturm count of
// that copy (one division per step); th[i] receives it.  The bisection stops
// at a relative bracket of 2^-30: the values only enter FP32 features.
__device__ inline void ritz_values(const double *al, const double *be, int m, double *d, double *e2, double *th) {
    const int j = threadIdx.x;
    if (j < m) {
        d[j] = 1.0 / al[j] + (j > 0 ? be[j - 1] / al[j - 1] : 0.0);
        e2[j] = j + 1 < m ? be[j] / (al[j] * al[j]) : 0.0;
    }
    __syncthreads();
    const int i = threadIdx.x;
    if (i < m) {
        double lo = INFINITY, up = -INFINITY;
        for (int k = 0; k < m; ++k) {
            const double r = (k > 0 ? sqrt(e2[k - 1]) : 0.0) + sqrt(e2[k]);
            lo = fmin(lo, d[k] - r);
            up = fmax(up, d[k] + r);
        }
        for (int it = 0; it < 128; ++it) {
            const double x = 0.5 * (lo + up);
            if (x <= lo || x >= up || up - lo <= 0x1p-30 * fmax(fabs(lo), fabs(up))) break;
            int cnt = 0;
            double q = 1.0;
            for (int k = 0; k < m; ++k) {
                q = (d[k] - x) - (k > 0 ? e2[k - 1] / q : 0.0);
                if (fabs(q) < 1e-300) q = -1e-300;
                cnt += q < 0.0;
            }
            if (cnt >= i + 1) up = x;
            else lo = x;
        }
        th[i] = 0.5 * (lo + up);
    }
    __syncthreads();
}

// The 16 features from the row statistics (RowStats order), the sum of
// squared deviations of ln d_i from their mean, the m sorted Ritz values
// th[0..m-1] and the relative residual after the steps.
__device__ inline void feature_vector(const double *st, double var, const double *th, int m, double relres, int32_t n,
                                      int64_t nnz, float *feat) {
    const double hi = st[1];
    const int top = m - 1;
    double f[16];
    f[0] = log10((double)n);
    f[1] = (double)nnz / (double)n;
    f[2] = st[0];
    f[3] = hi;
    f[4] = (st[3] - st[2]) / log(10.0);
    f[5] = sqrt(var / (double)n);
    f[6] = st[6] > 0.0 ? st[5] / st[6] : 0.0;
    // k-th smallest / largest Ritz values; with fewer than three, the index
    // clamps to the values that exist
    for (int k = 0; k < 3; ++k) {
        f[7 + k] = th[k < top ? k : top] / hi;
        f[10 + k] = th[top - 2 + k > 0 ? top - 2 + k : 0] / hi;
    }
    f[13] = log10(th[top] / th[0]);
    f[14] = log10(fmax(relres, 1e-30));  // floored: exact early convergence stays finite
    f[15] = log10(th[0] / hi);
    for (int k = 0; k < 16; ++k) feat[k] = (float)f[k];
}

// Row sum of a sliced-diagonal matrix (the layout of the SDIA schedule:
// offset/mask slots s*W .. s*W+W-1, value slots s*U .. s*U+U-1 of 64 lanes
// each): sum over the entries of row `row` in offset (column) order of
// fma(a_ij, u(j), sum).  Every active lane of the calling wavefront must hold
// a row of the same 64-row slice; rows >= n contribute nothing (their masks
// are 0).  All loads are issued unconditionally at in-bounds addresses.
// UC <= W: the slots walked, a compile-time bound >= the matrix's U (slots
// past U hold no entry in any slice).
template <int W, int UC = W, typename F>
__device__ __forceinline__ double sdia_row(const int32_t *__restrict__ soff, const uint64_t *__restrict__ smask,
                                           const double *__restrict__ sval, int U, int64_t n, int64_t row, F u) {
    const int64_t sl = __builtin_amdgcn_readfirstlane((int)(row >> 6));
    const int lane = (int)(row & 63);
    const int32_t *o = soff + sl * W;
    const uint64_t *m = smask + sl * W;
    const double *v = sval + sl * U * 64 + lane;
    const int rc = (int)(row < n ? row : n - 1);
    double a[W], g[W];
    bool in[W];
#pragma unroll
    for (int k = 0; k < UC; ++k) {
        const int ok = o[k];
        const uint64_t mk = m[k];
        a[k] = __builtin_nontemporal_load(v + (int64_t)(k < U ? k : U - 1) * 64);
        in[k] = (mk >> lane) & 1ull;
        g[k] = u(in[k] ? (int)row + ok : rc);
    }
    double sum = 0.0;
#pragma unroll
    for (int k = 0; k < UC; ++k) {
        const double t = fma(a[k], g[k], sum);
        sum = in[k] ? t : sum;
    }
    return sum;
}

// Pointers into the constant address space: loads through them are scalar
// (one per wavefront, into SGPRs).  Only for tables no kernel writes while
// the reading kernel runs.
using kc32 = const __attribute__((address_space(4))) int32_t;
using kc64 = const __attribute__((address_space(4))) uint64_t;

// Pointers into the global address space.  A pointer read from memory (a
// batch's per-system table) is generic, and loads through it are flat
// instructions, which count in lgkmcnt as well as vmcnt: waiting for a
// scalar load would then also wait for every vector load in flight.  Through
// these the loads and stores are global ones.
template <class T>
using glob_t = __attribute__((address_space(1))) T;
template <class T>
__device__ __forceinline__ glob_t<T> *glb(T *p) {
    return (glob_t<T> *)p;
}
template <class T>
__device__ __forceinline__ const glob_t<T> *glb(const T *p) {
    return (const glob_t<T> *)p;
}

// The rows of slices sl_begin, sl_begin + step, ... < sl_end of a matrix's
// sliced-diagonal copy (8 offset slots per slice, UC <= 8 walked), walked by
// one wavefront: for each slice, f(sl, row, rc, sum) with sum = sum_k a_k
// u(j_k) over the row's entries (column order, one FMA each: the sums of
// sdia_row) and rc = min(row, n - 1).  Offsets and masks are scalar loads;
// the gathers read row + offset clamped into [0, n) (an absent entry's
// product is dropped by a select on the mask, which is only needed then),
// and the next slice's values are loaded while the current slice's gathers
// are in flight.  sl must be uniform across the wavefront.
// SYM (the copy's value-symmetry flag set): an entry left of the diagonal,
// (i, i - q), is read as its transpose (i - q, i) from row i - q's slot of
// offset +q, whose index the copy's partner table holds (the table follows
// the offsets; low byte for the lanes whose transpose lies q/64 slices back,
// next byte for the lanes one slice further back), so only the slots on and
// right of the diagonal stream from memory and the others are lines read a
// few slices earlier.  Those addresses need the next slice's offsets, so
// the next values are issued after the current gathers, once the offsets
// (requested before the gathers) are in.  Same bits, so the same sums.
template <int UC, bool SYM = false, typename FU, typename FF>
__device__ __forceinline__ void sdia_slices(const int32_t *__restrict__ soff, const uint64_t *__restrict__ smask,
                                            const double *__restrict__ sval, int U, int64_t n, int sl_begin,
                                            int sl_end, int step, FU u, FF f) {
    const int lane = threadIdx.x & 63;
    const int64_t nsl = (n + 63) >> 6;
    const int nm1 = (int)n - 1;
    const glob_t<double> *sv = glb(sval);
    int on[UC], qn[UC];
    double an[UC];
    auto offs = [&](int sl) {
        const kc32 *o = (const kc32 *)(soff + (int64_t)sl * 8);
        const kc32 *q = (const kc32 *)(soff + (nsl + sl) * 8);
#pragma unroll
        for (int k = 0; k < UC; ++k) {
            on[k] = o[k];
            if constexpr (SYM) qn[k] = q[k];
        }
    };
    auto vals = [&](int sl) {
        const glob_t<double> *v = sv + (int64_t)sl * U * 64 + lane;
#pragma unroll
        for (int k = 0; k < UC; ++k) {
            if constexpr (SYM) {
                // own slot, or the transpose's: row + offset left of the
                // diagonal, clamped at 0 for an absent entry (any slot of a
                // slice at or before this one is a valid address; its value
                // is dropped); bit arithmetic, no branch per slot, so the
                // slice's loads stay one straight-line batch
                const int lowm = on[k] >> 31;  // all ones left of the diagonal
                const int r = max(sl * 64 + lane + (on[k] & lowm), 0);
                const int ps = (lane >= ((-on[k]) & 63) ? qn[k] : (qn[k] >> 8)) & 0xff;
                const int slot = (ps & lowm) | ((k < U ? k : U - 1) & ~lowm);
                an[k] = sv[((int64_t)(r >> 6) * U + slot) * 64 + (r & 63)];
            } else {
                an[k] = __builtin_nontemporal_load(v + (int64_t)(k < U ? k : U - 1) * 64);
            }
        }
    };
    if (sl_begin < sl_end) {
        offs(sl_begin);
        vals(sl_begin);
    }
    for (int sl = sl_begin; sl < sl_end; sl += step) {
        int oc[UC];
        double ac[UC];
        uint64_t mc[UC];
        const kc64 *m = (const kc64 *)(smask + (int64_t)sl * 8);
#pragma unroll
        for (int k = 0; k < UC; ++k) {
            oc[k] = on[k];
            ac[k] = an[k];
            mc[k] = m[k];
        }
        const bool more = sl + step < sl_end;
        if (more) {
            offs(sl + step);
            if constexpr (!SYM) vals(sl + step);  // in flight during the gathers below
        }
        const int row = sl * 64 + lane;
        const int rc = row < n ? row : nm1;
        double g[UC];
#pragma unroll
        for (int k = 0; k < UC; ++k) g[k] = u(min(max(row + oc[k], 0), nm1));
        if constexpr (SYM) {
            if (more) vals(sl + step);
        }
        double sum = 0.0;
#pragma unroll
        for (int k = 0; k < UC; ++k) {
            const double t = fma(ac[k], g[k], sum);
            sum = ((mc[k] >> lane) & 1ull) ? t : sum;
        }
        f(sl, row, rc, sum);
    }
}

// Whether a sliced-diagonal copy with 8 offset slots per slice may be read
// with its transposes (the value-symmetry flag after the partner table).
__device__ __forceinline__ bool sdia_sym8(const int32_t *soff, int64_t n) {
    return *(const kc32 *)(soff + ((n + 63) >> 6) * 16) != 0;
}

// A matrix as the row-per-thread kernels read it: the CSR arrays, and the
// sliced-diagonal copy when there is one.
struct RowMat {
    const int32_t *rowptr, *col;
    const double *val;
    const int32_t *soff;
    const uint64_t *smask;
    const double *sval;
    int U;
};

// sum_j a_ij u(j) of row i, entries in column-storage order with one FMA
// each: L = 0 reads the CSR arrays (rows of up to 8 entries issue every
// gather before the first FMA), L = 8/16/32 the sliced-diagonal copy of that
// slot width, L = 5/7 the 8-wide copy walking 5/7 slots (U <= L) (then each
// wavefront's rows must be one 64-row slice).
template <int L, typename F>
__device__ __forceinline__ double mat_row(const RowMat &M, int64_t n, int64_t i, F u) {
    if constexpr (L > 0) {
        return sdia_row<(L < 8 ? 8 : L), L>(M.soff, M.smask, M.sval, M.U, n, i, u);
    } else {
        const int s = M.rowptr[i], e = M.rowptr[i + 1];
        const int len = e - s;
        double sum = 0.0;
        if (len <= 8) {
            int jj[8];
            double aa[8], uj[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const bool in = q < len;
                jj[q] = in ? M.col[s + q] : (int)i;
                aa[q] = in ? M.val[s + q] : 0.0;
            }
#pragma unroll
            for (int q = 0; q < 8; ++q) uj[q] = u(jj[q]);
#pragma unroll
            for (int q = 0; q < 8; ++q)
                if (q < len) sum = fma(aa[q], uj[q], sum);
        } else {
            for (int k = s; k < e; ++k) sum = fma(M.val[k], u(M.col[k]), sum);
        }
        return sum;
    }
}

}  // namespace dev
}  // namespace apcg
