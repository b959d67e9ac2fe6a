// TFQMR (transpose-free QMR), the paper's second benchmark method (Section 4,
// "Transpose-Free Quasi-Minimal Residual"; Freund, SIAM J. Sci. Comput. 14,
// 1993), in the arrangement with two products per iteration, applied to the
// left-preconditioned system B A x = B b with B = D^{-1} (Jacobi) or I.
// Device-resident like the PCG path: every scalar lives in a small state
// record on the device, reductions are per-workgroup partials re-added in a
// fixed order by every workgroup of the next kernel, the host only paces
// K-iteration graphs and polls a flag.
//
// One iteration k (parity p = k & 1) is four kernels, one global reduction
// each:
//   A  sigma = r0.v -> alpha;  y2 = y1 - alpha v (formed in the gather),
//      u2 = B A y2;  half-step 1: w -= alpha u1, d = y1 + (theta^2 eta/alpha) d,
//      partials of ||w||^2
//   B  theta, c, tau, eta of half-step 1 and its test;  x += eta d;
//      half-step 2: w -= alpha u2, d = y2 + (theta^2 eta/alpha) d, ||w||^2
//   C  theta, c, tau, eta of half-step 2 and its test;  x += eta d;
//      partials of r0.w
//   D  rho' = r0.w -> beta;  y1 = w + beta y2 (formed in the gather),
//      u1 = B A y1;  v = u1 + beta (u2 + beta v);  partials of r0.v
// A test that stops the solve after an x update is recorded (stop_b by B,
// stop_c by C) and acted on by the next kernel, so every workgroup of the
// kernel that found it still applies its x update; B and C record in
// different fields because C reads B's.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <vector>

#include "internal.h"

namespace apcg {
namespace {

constexpr int TBQ = 256;
// slices of the context's partials buffer (kMaxBlocks doubles each)
constexpr int Q_INIT = 0, Q_SIG = 1, Q_W1 = 2, Q_W2 = 3, Q_RHO = 4;

void tq_grid(int64_t n, int *G, int64_t *per_block) {
    *G = normalise_blocks(1024, (n + 63) / 64);
    const int64_t pb = (n + *G - 1) / *G;
    *per_block = std::max<int64_t>(64, ((pb + 63) / 64) * 64);
}

struct TqHalf {
    double tau, theta, eta;
};

// Fields a kernel writes are never read by the same kernel: alpha, rho and
// the iteration count alternate by iteration parity, the half-step scalars
// by half-step (h[1] after half-step 1, h[0] after half-step 2).
struct TqState {
    double ref, rtol;
    double rho[2];
    double alpha[2];
    TqHalf h[2];
    double bound;  // tau sqrt(m + 1) of the last half-step
    int32_t its[2];
    int32_t half;
    int32_t maxit;
    int32_t status, flag, stop_b, stop_c;
};
static_assert(sizeof(TqState) <= 512, "TFQMR state exceeds its allocation");

using TqMat = dev::RowMat;

__device__ __forceinline__ void set_stop(TqState *st, int status) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        st->status = status;
        st->flag = 1;
    }
}

// B = D^{-1} (or I), r0 = B (b - A x0), w = y1 = r0, d = 0; partials of
// ||r0||^2 and of the count of unusable diagonal entries.
__global__ __launch_bounds__(TBQ) void k_tq_init(int32_t n, const int32_t *__restrict__ rowptr,
                                                 const int32_t *__restrict__ col, const double *__restrict__ val,
                                                 const double *__restrict__ b, double *__restrict__ x,
                                                 double *__restrict__ bd, double *__restrict__ r0,
                                                 double *__restrict__ w, double *__restrict__ y1,
                                                 double *__restrict__ d, double *part, int64_t per_block, int x0_zero,
                                                 int pc) {
    const dev::Chunk c = dev::block_chunk(n, per_block);
    double v[2] = {0.0, 0.0};
    for (int64_t i = c.lo + threadIdx.x; i < c.hi; i += TBQ) {
        double a = 0.0, ax = 0.0;
        bool found = false;
        for (int k = rowptr[i]; k < rowptr[i + 1]; ++k) {
            const int j = col[k];
            if (j == (int)i) {
                a = val[k];
                found = true;
            }
            if (!x0_zero) ax = fma(val[k], x[j], ax);
        }
        const bool ok = pc == APCG_PC_NONE || (found && a != 0.0 && isfinite(a));
        v[1] += ok ? 0.0 : 1.0;
        const double bi = pc == APCG_PC_NONE ? 1.0 : (ok ? 1.0 / a : 0.0);
        const double ri = bi * (x0_zero ? b[i] : b[i] - ax);
        bd[i] = bi;
        r0[i] = ri;
        w[i] = ri;
        y1[i] = ri;
        d[i] = 0.0;
        v[0] = fma(ri, ri, v[0]);
    }
    dev::store_partials<TBQ, 2>(v, part + (size_t)Q_INIT * kMaxBlocks, gridDim.x,
                                dev::xcd_block(blockIdx.x, gridDim.x));
}

__global__ __launch_bounds__(64) void k_tq_init_final(TqState *st, const double *part, int G, double rtol,
                                                      int32_t maxit) {
    double v[2];
    dev::reduce_partials<64, 2>(part + (size_t)Q_INIT * kMaxBlocks, G, v);
    if (threadIdx.x != 0) return;
    TqState s;
    s.ref = sqrt(v[0]);
    s.rtol = rtol;
    s.rho[0] = v[0];
    s.rho[1] = 0.0;
    s.alpha[0] = s.alpha[1] = 0.0;
    s.h[0] = TqHalf{s.ref, 0.0, 0.0};
    s.h[1] = s.h[0];
    s.bound = s.ref;
    s.its[0] = s.its[1] = 0;
    s.half = 0;
    s.maxit = maxit;
    s.stop_b = s.stop_c = 0;
    int status = 0;
    if (v[1] > 0.0) status = APCG_SOLVE_SETUP_ERROR;
    else if (!isfinite(s.ref)) status = APCG_SOLVE_NAN;
    else if (s.ref == 0.0) {
        status = APCG_SOLVE_CONVERGED;
        s.bound = 0.0;
    } else if (maxit <= 0) status = APCG_SOLVE_MAXIT;
    s.status = status;
    s.flag = status != 0;
    *st = s;
}

// u1 = B A y1, v = u1 and the partials of r0.v (sigma of iteration 1).
template <int L>
__global__ __launch_bounds__(TBQ) void k_tq_init_product(int32_t n, TqMat M,
                                                         const double *__restrict__ bd, const double *__restrict__ r0,
                                                         const double *__restrict__ y1, double *__restrict__ u1,
                                                         double *__restrict__ v, const TqState *st, double *part,
                                                         int64_t per_block) {
    if (st->flag) return;
    const dev::Chunk c = dev::block_chunk(n, per_block);
    double s[1] = {0.0};
    for (int64_t i = c.lo + threadIdx.x; i < c.hi; i += TBQ) {
        const double ui = bd[i] * dev::mat_row<L>(M, n, i, [&](int q) { return y1[q]; });
        u1[i] = ui;
        v[i] = ui;
        s[0] = fma(r0[i], ui, s[0]);
    }
    dev::store_partials<TBQ, 1>(s, part + (size_t)Q_SIG * kMaxBlocks, gridDim.x,
                                dev::xcd_block(blockIdx.x, gridDim.x));
}

// Kernel A of iteration (parity p).
template <int L>
__global__ __launch_bounds__(TBQ) void k_tq_a(int32_t n, TqMat M, const double *__restrict__ bd,
                                              const double *__restrict__ y1,
                                              const double *__restrict__ v, const double *__restrict__ u1,
                                              double *__restrict__ y2, double *__restrict__ u2,
                                              double *__restrict__ w, double *__restrict__ d, TqState *st, int p,
                                              double *part, int64_t per_block) {
    if (st->flag) return;
    double sg[1];
    dev::reduce_partials<TBQ, 1>(part + (size_t)Q_SIG * kMaxBlocks, gridDim.x, sg);
    const double sigma = sg[0];
    if (!isfinite(sigma)) return set_stop(st, APCG_SOLVE_NAN);
    if (sigma == 0.0) return set_stop(st, APCG_SOLVE_BREAKDOWN_PAP);
    const double alpha = st->rho[p ^ 1] / sigma;
    const TqHalf h = st->h[0];
    const double f = h.theta * h.theta * h.eta / alpha;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        st->alpha[p] = alpha;
        st->its[p] = st->its[p ^ 1] + 1;
    }
    const dev::Chunk c = dev::block_chunk(n, per_block);
    double s[1] = {0.0};
    for (int64_t i = c.lo + threadIdx.x; i < c.hi; i += TBQ) {
        const double ui = bd[i] * dev::mat_row<L>(M, n, i, [&](int q) { return fma(-alpha, v[q], y1[q]); });
        y2[i] = fma(-alpha, v[i], y1[i]);
        u2[i] = ui;
        const double wi = fma(-alpha, u1[i], w[i]);
        w[i] = wi;
        d[i] = fma(f, d[i], y1[i]);
        s[0] = fma(wi, wi, s[0]);
    }
    dev::store_partials<TBQ, 1>(s, part + (size_t)Q_W1 * kMaxBlocks, gridDim.x,
                                dev::xcd_block(blockIdx.x, gridDim.x));
}

// theta, c, tau, eta of a half-step from the reduced ||w||^2; the test of
// half-step m; returns the status the half-step ends the solve with (0:
// none).  Workgroup 0 records the scalars in h[slot].
__device__ int tq_half_step(TqState *st, const double *part, int G, double tau_prev, double alpha, int m,
                            int slot, TqHalf *out) {
    double ww[1];
    dev::reduce_partials<TBQ, 1>(part, G, ww);
    const double theta = sqrt(ww[0]) / tau_prev;
    const double cc = 1.0 / sqrt(1.0 + theta * theta);
    const TqHalf h{tau_prev * theta * cc, theta, cc * cc * alpha};
    const double bound = h.tau * sqrt((double)m + 1.0);
    int status = 0;
    if (!isfinite(bound)) status = APCG_SOLVE_NAN;
    else if (bound <= st->rtol * st->ref) status = APCG_SOLVE_CONVERGED;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        st->h[slot] = h;
        st->bound = bound;
        st->half = m;
    }
    *out = h;
    return status;
}

// Kernel B of iteration (parity p).
__global__ __launch_bounds__(TBQ) void k_tq_b(int64_t n, double *__restrict__ x, double *__restrict__ d,
                                              double *__restrict__ w, const double *__restrict__ u2,
                                              const double *__restrict__ y2, TqState *st, int p, double *part,
                                              int64_t per_block) {
    if (st->flag) return;
    const double alpha = st->alpha[p];
    const int k = st->its[p];
    TqHalf h;
    const int status =
        tq_half_step(st, part + (size_t)Q_W1 * kMaxBlocks, gridDim.x, st->h[0].tau, alpha, 2 * k - 1, 1, &h);
    if (status && blockIdx.x == 0 && threadIdx.x == 0) st->stop_b = status;
    const double f = h.theta * h.theta * h.eta / alpha;
    const dev::Chunk c = dev::block_chunk(n, per_block);
    double s[1] = {0.0};
    for (int64_t i = c.lo + threadIdx.x; i < c.hi; i += TBQ) {
        const double di = d[i];
        x[i] = fma(h.eta, di, x[i]);
        if (status) continue;
        const double wi = fma(-alpha, u2[i], w[i]);
        w[i] = wi;
        d[i] = fma(f, di, y2[i]);
        s[0] = fma(wi, wi, s[0]);
    }
    if (status) return;
    dev::store_partials<TBQ, 1>(s, part + (size_t)Q_W2 * kMaxBlocks, gridDim.x,
                                dev::xcd_block(blockIdx.x, gridDim.x));
}

// A test recorded by the previous kernel ends the solve here.
__device__ __forceinline__ bool tq_pending(TqState *st, int pending) {
    if (pending) set_stop(st, pending);
    return pending != 0;
}

// Kernel C of iteration (parity p).
__global__ __launch_bounds__(TBQ) void k_tq_c(int64_t n, double *__restrict__ x, const double *__restrict__ d,
                                              const double *__restrict__ w, const double *__restrict__ r0,
                                              TqState *st, int p, double *part, int64_t per_block) {
    if (st->flag || tq_pending(st, st->stop_b)) return;
    const double alpha = st->alpha[p];
    const int k = st->its[p];
    TqHalf h;
    int status = tq_half_step(st, part + (size_t)Q_W2 * kMaxBlocks, gridDim.x, st->h[1].tau, alpha, 2 * k, 0, &h);
    if (!status && k >= st->maxit) status = APCG_SOLVE_MAXIT;
    if (status && blockIdx.x == 0 && threadIdx.x == 0) st->stop_c = status;
    const dev::Chunk c = dev::block_chunk(n, per_block);
    double s[1] = {0.0};
    for (int64_t i = c.lo + threadIdx.x; i < c.hi; i += TBQ) {
        x[i] = fma(h.eta, d[i], x[i]);
        s[0] = fma(r0[i], w[i], s[0]);
    }
    if (status) return;
    dev::store_partials<TBQ, 1>(s, part + (size_t)Q_RHO * kMaxBlocks, gridDim.x,
                                dev::xcd_block(blockIdx.x, gridDim.x));
}

// Kernel D of iteration (parity p).
template <int L>
__global__ __launch_bounds__(TBQ) void k_tq_d(int32_t n, TqMat M, const double *__restrict__ bd,
                                              const double *__restrict__ r0,
                                              const double *__restrict__ w, const double *__restrict__ y2,
                                              const double *__restrict__ u2, double *__restrict__ y1,
                                              double *__restrict__ u1, double *__restrict__ v, TqState *st, int p,
                                              double *part, int64_t per_block) {
    if (st->flag || tq_pending(st, st->stop_c)) return;
    double rr[1];
    dev::reduce_partials<TBQ, 1>(part + (size_t)Q_RHO * kMaxBlocks, gridDim.x, rr);
    const double rho = rr[0];
    if (!isfinite(rho)) return set_stop(st, APCG_SOLVE_NAN);
    if (rho == 0.0) return set_stop(st, APCG_SOLVE_BREAKDOWN_RZ);
    const double beta = rho / st->rho[p ^ 1];
    if (blockIdx.x == 0 && threadIdx.x == 0) st->rho[p] = rho;
    const dev::Chunk c = dev::block_chunk(n, per_block);
    double s[1] = {0.0};
    for (int64_t i = c.lo + threadIdx.x; i < c.hi; i += TBQ) {
        const double ui = bd[i] * dev::mat_row<L>(M, n, i, [&](int q) { return fma(beta, y2[q], w[q]); });
        y1[i] = fma(beta, y2[i], w[i]);
        u1[i] = ui;
        const double vi = fma(beta, fma(beta, v[i], u2[i]), ui);
        v[i] = vi;
        s[0] = fma(r0[i], vi, s[0]);
    }
    dev::store_partials<TBQ, 1>(s, part + (size_t)Q_SIG * kMaxBlocks, gridDim.x,
                                dev::xcd_block(blockIdx.x, gridDim.x));
}

__global__ void k_tq_finish(const TqState *st, apcg_solve_info *out) {
    if (threadIdx.x != 0) return;
    int status = st->status;
    if (!status) status = st->stop_c ? st->stop_c : (st->stop_b ? st->stop_b : APCG_SOLVE_MAXIT);
    apcg_solve_info o;
    o.iterations = std::max(st->its[0], st->its[1]);
    o.status = status;
    o.fcg_iterations = 0;
    o.half_steps = st->half;
    o.res_norm = st->bound;
    o.ref_norm = st->ref;
    *out = o;
}

struct TqCache {
    int device = 0;
    int64_t cap = 0;
    double *ws = nullptr;  // 9 * cap: bd, r0, w, y1, y2, u1, u2, v, d
    TqState *st = nullptr;
    int32_t *pinned = nullptr;  // (status, flag) per lookahead slot
    EventRef poll_ev[kMaxLookahead];
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    const void *gkey[11] = {};
    int32_t gK = 0;
};

}  // namespace

static std::mutex g_tq_mu;
static std::vector<std::pair<uint64_t, TqCache *>> g_tq;

static TqCache *tq_cache(apcg_ctx c) {
    std::lock_guard<std::mutex> lk(g_tq_mu);
    for (auto &p : g_tq)
        if (p.first == c->id) return p.second;
    TqCache *s = new TqCache();
    s->device = c->device;
    g_tq.emplace_back(c->id, s);
    return s;
}

void tq_cache_release(uint64_t ctx_id, int device) {
    TqCache *s = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_tq_mu);
        for (auto it = g_tq.begin(); it != g_tq.end(); ++it)
            if (it->first == ctx_id) {
                s = it->second;
                g_tq.erase(it);
                break;
            }
    }
    if (!s) return;
    hipSetDevice(device);
    if (s->exec) hipGraphExecDestroy(s->exec);
    if (s->graph) hipGraphDestroy(s->graph);
    hipFree(s->ws);
    hipFree(s->st);
    if (s->pinned) hipHostFree(s->pinned);
    delete s;
}

}  // namespace apcg

using namespace apcg;

extern "C" apcg_status apcg_ksp_solve_tfqmr(apcg_ctx ctx, apcg_mat A, apcg_vec b, apcg_vec x, double rtol,
                                            int32_t maxit, const apcg_solve_opts *opts_in, apcg_info info,
                                            int32_t info_index) {
    try {
        if (!ctx || !A || !b || !x || !info) return set_error(APCG_ERR_INVALID_ARG, "NULL argument");
        if (b->n != A->n || x->n != A->n) return set_error(APCG_ERR_INVALID_ARG, "dimension mismatch");
        if (vec_overlap(b, x)) return set_error(APCG_ERR_INVALID_ARG, "b and x must not share memory");
        if (ctx->device != A->device || b->device != A->device || x->device != A->device ||
            info->device != A->device)
            return set_error(APCG_ERR_INVALID_ARG, "operands on different devices");
        if (info_index < 0 || info_index >= info->count)
            return set_error(APCG_ERR_INVALID_ARG, "info index out of range");
        if (!(rtol >= 0.0) || !std::isfinite(rtol)) return set_error(APCG_ERR_INVALID_ARG, "rtol must be finite and >= 0");
        if (maxit < 0) return set_error(APCG_ERR_INVALID_ARG, "maxit must be >= 0");
        if (ctx->type == APCG_STREAM_GLOBAL_BLOCKING && ctx->is_default_global)
            return set_error(APCG_ERR_INVALID_ARG, "pass a context created with apcg_ctx_create");
        apcg_solve_opts opts;
        if (opts_in) opts = *opts_in;
        else apcg_solve_opts_default(&opts);
        if (opts.pc != APCG_PC_NONE && opts.pc != APCG_PC_JACOBI)
            return set_error(APCG_ERR_INVALID_ARG, "unknown preconditioner");
        if (opts.mode < APCG_MODE_GRAPH || opts.mode > APCG_MODE_HOST_CHECK)
            return set_error(APCG_ERR_INVALID_ARG, "unknown mode");
        if (opts.iters_per_graph < 1) return set_error(APCG_ERR_INVALID_ARG, "iters_per_graph must be >= 1");
        if (opts.lookahead < 1 || opts.lookahead > kMaxLookahead)
            return set_error(APCG_ERR_INVALID_ARG, "lookahead must be in [1, 8]");
        int K = std::max(2, opts.iters_per_graph);
        if (K & 1) ++K;  // even: the parities of a period match the global iterations'
        const int L = opts.lookahead;
        const bool host_check = opts.mode == APCG_MODE_HOST_CHECK;

        TqCache *tc = tq_cache(ctx);
        const int dev = ctx->device;
        hipStream_t st = ctx->stream;
        Acc acc[4] = {{&x->rec, ACC_RW}, {&info->rec, ACC_W}, {&A->rec, ACC_R}, {&b->rec, ACC_R}};
        apcg_status s;
        if ((s = op_begin(ctx, acc, 4))) return s;
        const int64_t n = A->n;
        if (tc->cap < n || !tc->ws) {
            if (tc->ws) {
                EventRef ev = event_get(dev);
                if (!ev) return set_error(APCG_ERR_HIP, "event creation failed");
                APCG_HIP(hipEventRecord(ev->e, st));
                double *old = tc->ws;
                hipGraphExec_t oe = tc->exec;
                hipGraph_t og = tc->graph;
                defer_release({ev}, [old, oe, og, dev]() {
                    hipSetDevice(dev);
                    if (oe) hipGraphExecDestroy(oe);
                    if (og) hipGraphDestroy(og);
                    hipFree(old);
                });
                tc->exec = nullptr;
                tc->graph = nullptr;
            }
            const int64_t cap = std::max<int64_t>(64, ((n + 63) / 64) * 64);
            APCG_HIP(hipMalloc((void **)&tc->ws, sizeof(double) * 9 * cap));
            tc->cap = cap;
        }
        if (!tc->st) {
            APCG_HIP(hipMalloc((void **)&tc->st, 512));
            APCG_HIP(hipHostMalloc((void **)&tc->pinned, sizeof(int32_t) * 2 * kMaxLookahead, hipHostMallocDefault));
        }
        const int64_t cap = tc->cap;
        double *bd = tc->ws, *r0 = tc->ws + cap, *w = tc->ws + 2 * cap, *y1 = tc->ws + 3 * cap;
        double *y2 = tc->ws + 4 * cap, *u1 = tc->ws + 5 * cap, *u2 = tc->ws + 6 * cap, *v = tc->ws + 7 * cap;
        double *d = tc->ws + 8 * cap;
        double *part = ctx->partials;
        int G;
        int64_t pb;
        tq_grid(n, &G, &pb);
        const int x0z = opts.x0_is_zero ? 1 : 0;
        // products on the sliced-diagonal copy whenever the pattern allows it
        // (the analysis is a one-time host pass per matrix; the sums are
        // bitwise those of the CSR rows)
        int lw = 0;  // slot width of the sliced-diagonal copy, 0: CSR
        if ((s = sdia_analyse(A))) return s;
        if (A->sdia_state == 1) {
            if ((s = prepare_sdia(A, st))) return s;
            lw = sdia_walk(A);
        }
        const TqMat M{A->rowptr, A->col, A->val, A->sdia_off, A->sdia_msk, A->sdia_val, A->sdia_u};
        auto sync_if = [&]() -> apcg_status {
            if (host_check) {
                g_counters.host_syncs++;
                APCG_HIP(hipStreamSynchronize(st));
            }
            return APCG_SUCCESS;
        };

        if (x0z && n > 0) APCG_HIP(hipMemsetAsync(x->d, 0, sizeof(double) * n, st));
        hipLaunchKernelGGL(k_tq_init, dim3(G), dim3(TBQ), 0, st, A->n, A->rowptr, A->col, A->val, b->d, x->d, bd, r0,
                           w, y1, d, part, pb, x0z, opts.pc);
        APCG_CHECK_LAUNCH("k_tq_init");
        hipLaunchKernelGGL(k_tq_init_final, dim3(1), dim3(64), 0, st, tc->st, (const double *)part, G, rtol, maxit);
        APCG_CHECK_LAUNCH("k_tq_init_final");
        {
            auto f = lw == 5 ? k_tq_init_product<5> : lw == 7 ? k_tq_init_product<7>
                   : lw == 8 ? k_tq_init_product<8> : lw == 16 ? k_tq_init_product<16>
                   : lw == 32 ? k_tq_init_product<32> : k_tq_init_product<0>;
            hipLaunchKernelGGL(f, dim3(G), dim3(TBQ), 0, st, A->n, M, (const double *)bd, (const double *)r0,
                               (const double *)y1, u1, v, (const TqState *)tc->st, part, pb);
            APCG_CHECK_LAUNCH("k_tq_init_product");
        }
        auto fa = lw == 5 ? k_tq_a<5> : lw == 7 ? k_tq_a<7> : lw == 8 ? k_tq_a<8> : lw == 16 ? k_tq_a<16>
                : lw == 32 ? k_tq_a<32> : k_tq_a<0>;
        auto fd = lw == 5 ? k_tq_d<5> : lw == 7 ? k_tq_d<7> : lw == 8 ? k_tq_d<8> : lw == 16 ? k_tq_d<16>
                : lw == 32 ? k_tq_d<32> : k_tq_d<0>;
        if ((s = sync_if())) return s;

        auto iteration = [&](int j) -> apcg_status {
            const int p = j & 1;
            hipLaunchKernelGGL(fa, dim3(G), dim3(TBQ), 0, st, A->n, M, (const double *)bd, (const double *)y1,
                               (const double *)v, (const double *)u1, y2, u2, w, d, tc->st, p, part, pb);
            APCG_CHECK_LAUNCH("k_tq_a");
            apcg_status e;
            if ((e = sync_if())) return e;
            hipLaunchKernelGGL(k_tq_b, dim3(G), dim3(TBQ), 0, st, n, x->d, d, w, (const double *)u2,
                               (const double *)y2, tc->st, p, part, pb);
            APCG_CHECK_LAUNCH("k_tq_b");
            if ((e = sync_if())) return e;
            hipLaunchKernelGGL(k_tq_c, dim3(G), dim3(TBQ), 0, st, n, x->d, (const double *)d, (const double *)w,
                               (const double *)r0, tc->st, p, part, pb);
            APCG_CHECK_LAUNCH("k_tq_c");
            if ((e = sync_if())) return e;
            hipLaunchKernelGGL(fd, dim3(G), dim3(TBQ), 0, st, A->n, M, (const double *)bd, (const double *)r0,
                               (const double *)w, (const double *)y2, (const double *)u2, y1, u1, v, tc->st, p, part,
                               pb);
            APCG_CHECK_LAUNCH("k_tq_d");
            return sync_if();
        };

        if (maxit > 0) {
            if (opts.mode == APCG_MODE_GRAPH) {
                const void *key[11] = {(const void *)(uintptr_t)A->uid, A->rowptr, A->col, A->val, x->d, tc->ws,
                                       (const void *)ctx->partials, (const void *)(intptr_t)n,
                                       (const void *)(intptr_t)opts.pc, (const void *)(intptr_t)lw, A->sdia_val};
                if (!tc->exec || tc->gK != K || memcmp(key, tc->gkey, sizeof key) != 0) {
                    if (tc->exec) {
                        EventRef ev = event_get(dev);
                        if (ev) hipEventRecord(ev->e, st);
                        hipGraphExec_t oe = tc->exec;
                        hipGraph_t og = tc->graph;
                        defer_release({ev}, [oe, og, dev]() {
                            hipSetDevice(dev);
                            hipGraphExecDestroy(oe);
                            hipGraphDestroy(og);
                        });
                        tc->exec = nullptr;
                        tc->graph = nullptr;
                    }
                    APCG_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeRelaxed));
                    apcg_status cs = APCG_SUCCESS;
                    for (int j = 1; j <= K && cs == APCG_SUCCESS; ++j) cs = iteration(j);
                    hipGraph_t g = nullptr;
                    hipError_t e = hipStreamEndCapture(st, &g);
                    if (cs) {
                        if (g) hipGraphDestroy(g);
                        return cs;
                    }
                    if (e != hipSuccess) return hip_error(e, "hipStreamEndCapture(tfqmr)");
                    g_counters.kernel_launches -= (int64_t)4 * K;
                    e = hipGraphInstantiate(&tc->exec, g, nullptr, nullptr, 0);
                    if (e != hipSuccess) {
                        hipGraphDestroy(g);
                        return hip_error(e, "hipGraphInstantiate(tfqmr)");
                    }
                    tc->graph = g;
                    memcpy(tc->gkey, key, sizeof key);
                    tc->gK = K;
                }
            }
            const int64_t periods = ((int64_t)maxit + K - 1) / K;
            for (int64_t g = 0; g < periods; ++g) {
                if (opts.mode == APCG_MODE_GRAPH) {
                    g_counters.graph_launches++;
                    APCG_HIP(hipGraphLaunch(tc->exec, st));
                } else {
                    for (int j = 1; j <= K; ++j)
                        if ((s = iteration(j))) return s;
                }
                const int slot = (int)(g % L);
                if (!tc->poll_ev[slot]) {
                    tc->poll_ev[slot] = event_get(dev);
                    if (!tc->poll_ev[slot]) return set_error(APCG_ERR_HIP, "event creation failed");
                }
                g_counters.d2h_copies++;
                APCG_HIP(hipMemcpyAsync(&tc->pinned[2 * slot], &tc->st->status, 2 * sizeof(int32_t),
                                        hipMemcpyDeviceToHost, st));
                APCG_HIP(hipEventRecord(tc->poll_ev[slot]->e, st));
                if (g >= L - 1) {
                    const int ps = (int)((g - (L - 1)) % L);
                    g_counters.host_polls++;
                    APCG_HIP(hipEventSynchronize(tc->poll_ev[ps]->e));
                    if (tc->pinned[2 * ps + 1]) break;  // flag
                }
            }
        }
        hipLaunchKernelGGL(k_tq_finish, dim3(1), dim3(64), 0, st, (const TqState *)tc->st, info->d + info_index);
        APCG_CHECK_LAUNCH("k_tq_finish");
        return op_end(ctx, acc, 4);
    } catch (const std::bad_alloc &) {
        return set_error(APCG_ERR_OUT_OF_MEMORY, "host allocation failed");
    }
}
