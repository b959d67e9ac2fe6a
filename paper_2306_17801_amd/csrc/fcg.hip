// fcg.hip -- flexible CG, FCG(1), with a degree-8 Chebyshev polynomial
// preconditioner, and its fallback to Jacobi-PCG.
//
// Preconditioner: z = P r = sum_{j=0..8} c_j T_j(Y) v with v = D^-1 r and
// Y = (2/lmax) D^-1 A - I (lmax = the Gershgorin upper bound of D^-1 A),
// evaluated by Clenshaw's recurrence b_j = c_j v + 2 Y b_{j+1} - b_{j+2}
// (b_9 = b_10 = 0), z = c_0 v + Y b_1 - b_2: eight products with A.  FCG(1)
// (Notay 2000; Golub & Ye 1999): the PCG loop of Section 3.3 with
// beta = -(z_{k+1} . w_k) / (p_k . w_k), which keeps the search directions
// A-orthogonal when P is applied inexactly (FP32-derived coefficients).
//
// One iteration is 10 kernels: product (p = z + beta p_old, w = A p, p.w),
// update (x, r, ||r||^2), and eight Clenshaw steps (the last forms z and
// r.z, z.w).  No scalar kernels: each kernel's workgroups re-add the
// previous kernel's per-workgroup partials in a fixed order and all obtain
// the same scalars (beta and the r.z breakdown test in the product, alpha
// and the p.w breakdown test in the update, the convergence / stall / maxit
// test in the first Clenshaw step); workgroup 0 records them in the state,
// and the stop flag makes every later kernel a no-op.
// Before the first iteration p is evaluated on 1024 points of [0, lmax]; a
// value <= 0 (the preconditioner would not be SPD) stops the flexible phase
// at once.  A breakdown, that rejection, or a stall (no new minimum of ||r||
// in the last max(stall_min, stall_frac * k) iterations) hands over to
// Jacobi-PCG from the current x when the fallback is enabled.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>

#include "internal.h"

namespace apcg {
namespace {

constexpr int TBF = 256;
constexpr int DEG = 8;
// slices of the context's partials buffer (kMaxBlocks doubles each)
constexpr int S_INIT = 0, S_DELTA = 1, S_RES = 2, S_RZ = 3;

// Workgroups and rows per workgroup of the FCG kernels: at most 1024
// workgroups, so that re-adding a kernel's partials stays short.
void fcg_grid(int64_t n, int *G, int64_t *per_block) {
    *G = normalise_blocks(1024, (n + 63) / 64);
    const int64_t pb = (n + *G - 1) / *G;
    *per_block = std::max<int64_t>(64, ((pb + 63) / 64) * 64);
}

// Per-iteration test state, double-buffered by iteration parity: the
// kernel that runs the test for iteration k reads record (k - 1) & 1 and
// writes record k & 1, so no workgroup reads what another workgroup of the
// same kernel writes.
struct FcgRec {
    double res, best_res;
    int32_t its, best_its;
};

struct FcgState {
    double c[DEG + 1];
    double lmax;
    double rho, delta, alpha, beta;
    double ref, rtol;
    double stall_frac;
    FcgRec rec[2];
    int32_t maxit, stall_min;
    int32_t status, flag, zero_x, reject;
};
static_assert(sizeof(FcgState) <= 448, "FCG state exceeds its allocation");
// The state's allocation is 512 bytes; the fallback gate (int32[2], written
// by k_fcg_gate) sits at this byte offset after it.
constexpr int kGateOffset = 448;

__device__ __forceinline__ double pdir_f(double z, double beta, double pold) { return fma(beta, pold, z); }

__global__ __launch_bounds__(TBF) void k_fcg_init(int32_t n, const int32_t *__restrict__ rowptr,
                                                  const int32_t *__restrict__ col, const double *__restrict__ val,
                                                  const double *__restrict__ b, double *__restrict__ x,
                                                  double *__restrict__ r, double *__restrict__ dinv,
                                                  double *__restrict__ pold, double *part, int64_t per_block,
                                                  int x0_zero) {
    const dev::Chunk c = dev::block_chunk(n, per_block);
    double v[3] = {0.0, 0.0, 0.0};  // ||b||^2, ||r||^2, bad diagonals
    for (int64_t i = c.lo + threadIdx.x; i < c.hi; i += TBF) {
        double d = 0.0, ax = 0.0;
        bool found = false;
        for (int k = rowptr[i]; k < rowptr[i + 1]; ++k) {
            const int j = col[k];
            if (j == (int)i) {
                d = val[k];
                found = true;
            }
            if (!x0_zero) ax = fma(val[k], x[j], ax);
        }
        const bool ok = found && d > 0.0;
        v[2] += ok ? 0.0 : 1.0;
        const double bi = b[i];
        const double ri = x0_zero ? bi : bi - ax;
        r[i] = ri;
        dinv[i] = ok ? 1.0 / d : 0.0;
        pold[i] = 0.0;
        if (x0_zero) x[i] = 0.0;
        v[0] = fma(bi, bi, v[0]);
        v[1] = fma(ri, ri, v[1]);
    }
    dev::store_partials<TBF, 3>(v, part, gridDim.x, dev::xcd_block(blockIdx.x, gridDim.x));
}

// Clenshaw evaluation of p at one point t (scalar).
__device__ double poly_at(const double *c, double t, double lmax) {
    const double y = 2.0 * t / lmax - 1.0;
    double b1 = 0.0, b2 = 0.0;
    for (int j = DEG; j >= 1; --j) {
        const double b0 = c[j] + 2.0 * y * b1 - b2;
        b2 = b1;
        b1 = b0;
    }
    return c[0] + y * b1 - b2;
}

__global__ __launch_bounds__(64) void k_fcg_init_final(FcgState *st, const double *part, int G, const float *coef,
                                                       const double *lmax, double rtol, int32_t maxit,
                                                       int32_t stall_min, double stall_frac) {
    double v[3];
    dev::reduce_partials<64, 3>(part, G, v);
    __shared__ double cc[DEG + 1];
    __shared__ int bad_point;
    if (threadIdx.x <= DEG) cc[threadIdx.x] = (double)coef[threadIdx.x];
    if (threadIdx.x == 0) bad_point = 0;
    __syncthreads();
    const double lm = *lmax;
    // positivity of p on [0, lmax]: 1024 points
    for (int q = threadIdx.x; q < 1024; q += 64)
        if (!(poly_at(cc, lm * q / 1023.0, lm) > 0.0)) atomicOr(&bad_point, 1);
    __syncthreads();
    if (threadIdx.x != 0) return;
    FcgState s;
    for (int j = 0; j <= DEG; ++j) s.c[j] = cc[j];
    s.lmax = lm;
    s.ref = sqrt(v[0]);
    const double res0 = sqrt(v[1]);
    s.rtol = rtol;
    s.stall_frac = stall_frac;
    for (int k = 0; k < 2; ++k) s.rec[k] = FcgRec{res0, res0, 0, 0};
    s.maxit = maxit;
    s.stall_min = stall_min;
    s.rho = s.delta = s.alpha = s.beta = 0.0;
    s.zero_x = 0;
    s.reject = 0;
    int status = 0;
    if (v[2] > 0.0) status = APCG_SOLVE_SETUP_ERROR;
    else if (s.ref == 0.0) {
        status = APCG_SOLVE_CONVERGED;
        s.zero_x = 1;
        s.rec[0].res = s.rec[1].res = 0.0;
    } else if (!isfinite(res0) || !isfinite(s.ref)) status = APCG_SOLVE_NAN;
    else if (res0 <= rtol * s.ref) status = APCG_SOLVE_CONVERGED;
    else if (bad_point || !(lm > 0.0) || !isfinite(lm)) {
        status = APCG_SOLVE_BREAKDOWN_RZ;  // the preconditioner is not positive on [0, lmax]
        s.reject = 1;
    } else if (maxit <= 0) status = APCG_SOLVE_MAXIT;
    s.status = status;
    s.flag = status != 0;
    *st = s;
}

__global__ __launch_bounds__(TBF) void k_fcg_zero_x_if(double *__restrict__ x, int64_t n, int64_t per_block,
                                                       const FcgState *st) {
    if (!st->zero_x) return;
    const dev::Chunk c = dev::block_chunk(n, per_block);
    for (int64_t i = c.lo + threadIdx.x; i < c.hi; i += TBF) x[i] = 0.0;
}

// Convergence, stall and iteration-cap test after an update, from the
// update's ||r||^2 partials (every workgroup decides alike; workgroup 0
// records).  Returns true when the solve stops.
__device__ bool fcg_check(FcgState *st, const double *part_res, int G, int parity) {
    double v[1];
    dev::reduce_partials<TBF, 1>(part_res, G, v);
    const double res = sqrt(v[0]);
    const FcgRec prev = st->rec[parity ^ 1];
    FcgRec cur{res, prev.best_res, prev.its + 1, prev.best_its};
    int status = 0;
    if (!isfinite(res)) status = APCG_SOLVE_NAN;
    else if (res <= st->rtol * st->ref) status = APCG_SOLVE_CONVERGED;
    else {
        if (res < cur.best_res) {
            cur.best_res = res;
            cur.best_its = cur.its;
        } else {
            double win = st->stall_frac * (double)cur.its;
            if (win < (double)st->stall_min) win = (double)st->stall_min;
            if ((double)(cur.its - cur.best_its) >= win) status = APCG_SOLVE_STALL;
        }
        if (!status && cur.its >= st->maxit) status = APCG_SOLVE_MAXIT;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        st->rec[parity] = cur;
        if (status) {
            st->status = status;
            st->flag = 1;
        }
    }
    return status != 0;
}

// Rows [ch.lo, ch.hi) of a workgroup (ch.lo a multiple of 64) as the
// row-per-thread loop visits them -- thread t takes rows ch.lo + t,
// ch.lo + t + TBF, ... -- with f(i, (A u)_i) for each row i < n.  L = 5/7/8
// (an 8-wide sliced-diagonal copy): each wavefront walks its slices with the
// next slice's loads in flight (dev::sdia_slices), reading the entries left
// of the diagonal as their transposes while the copy's values are
// symmetric; otherwise dev::mat_row.  Same sums, same order, same bits.
template <int L, typename FU, typename FF>
__device__ __forceinline__ void fcg_rows(int32_t n, const dev::RowMat &M, dev::Chunk ch, FU u, FF f) {
    if constexpr (L == 5 || L == 7 || L == 8) {
        const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
        const int sb = (int)(ch.lo >> 6) + wave, se = (int)((ch.hi + 63) >> 6);
        auto g = [&](int, int row, int, double a) {
            if (row < n) f((int64_t)row, a);
        };
        if (dev::sdia_sym8(M.soff, n)) dev::sdia_slices<L, true>(M.soff, M.smask, M.sval, M.U, n, sb, se, TBF / 64, u, g);
        else dev::sdia_slices<L>(M.soff, M.smask, M.sval, M.U, n, sb, se, TBF / 64, u, g);
    } else {
        for (int64_t i = ch.lo + threadIdx.x; i < ch.hi; i += TBF) f(i, dev::mat_row<L>(M, n, i, u));
    }
}

// One Clenshaw step.  stage: 0 = first (j = DEG-1), 1 = middle, 2 = last
// (forms z and the partials of r.z and z.w).  check != 0 (inside the
// iteration): the first step first runs the test above for the iteration of
// the given parity.
// L: 0 = CSR products, 5/7/8/16/32 = the sliced-diagonal copy.
template <int L>
__global__ __launch_bounds__(TBF) void k_cheb(int32_t n, dev::RowMat M,
                                              const double *__restrict__ r, const double *__restrict__ dinv,
                                              const double *__restrict__ bj1, const double *__restrict__ bj2,
                                              double *__restrict__ out, const double *__restrict__ w,
                                              FcgState *st, int j, int stage, int check, int parity,
                                              double *partials, int64_t per_block) {
    if (st->flag) return;
    if (check && fcg_check(st, partials + (size_t)S_RES * kMaxBlocks, gridDim.x, parity)) return;
    const double s2 = 2.0 / st->lmax;
    const double cj = st->c[j], cd = st->c[DEG];
    const dev::Chunk ch = dev::block_chunk(n, per_block);
    double v[2] = {0.0, 0.0};
    if (stage == 0) {  // b_{d-1} = c_{d-1} v + 2 c_d Y v
        fcg_rows<L>(n, M, ch, [&](int q) { return dinv[q] * r[q]; }, [&](int64_t i, double av) {
#pragma clang fp contract(off)
            const double vi = dinv[i] * r[i];
            const double yv = s2 * dinv[i] * av - vi;
            out[i] = fma(2.0 * cd, yv, cj * vi);
        });
    } else {
        fcg_rows<L>(n, M, ch, [&](int q) { return bj1[q]; }, [&](int64_t i, double au) {
#pragma clang fp contract(off)
            const double vi = dinv[i] * r[i];
            const double yu = s2 * dinv[i] * au - bj1[i];
            const double b2v = bj2 ? bj2[i] : cd * vi;  // b_{d} = c_d v is not stored
            double res;
            if (stage == 1) res = fma(2.0, yu, cj * vi) - b2v;
            else {
                res = cj * vi + yu - b2v;
                v[0] = fma(r[i], res, v[0]);
                v[1] = fma(res, w[i], v[1]);
            }
            out[i] = res;
        });
    }
    if (stage == 2)
        dev::store_partials<TBF, 2>(v, partials + (size_t)S_RZ * kMaxBlocks, gridDim.x,
                                    dev::xcd_block(blockIdx.x, gridDim.x));
}

// p = z + beta p_old, w = A p and the partials of p.w.  Prologue: r.z and
// z.w of the last preconditioner application give rho and, after the first
// iteration, beta = -(z.w) / delta_prev (FCG(1)); r.z <= 0 is a breakdown.
template <int L>
__global__ __launch_bounds__(TBF) void k_fcg_product(int32_t n, dev::RowMat M,
                                                     const double *__restrict__ z, const double *__restrict__ pold,
                                                     double *__restrict__ pnew, double *__restrict__ w,
                                                     FcgState *st, int parity, double *partials,
                                                     int64_t per_block) {
    if (st->flag) return;
    double rz[2];
    dev::reduce_partials<TBF, 2>(partials + (size_t)S_RZ * kMaxBlocks, gridDim.x, rz);
    // no iteration done yet: z.w of the first application is not used (w unset)
    const bool first = st->rec[parity ^ 1].its == 0;
    int status = 0;
    double beta = 0.0;
    if (!isfinite(rz[0]) || (!first && !isfinite(rz[1]))) status = APCG_SOLVE_NAN;
    else if (!(rz[0] > 0.0)) status = APCG_SOLVE_BREAKDOWN_RZ;
    else if (!first) beta = -rz[1] / st->delta;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        if (status) {
            st->status = status;
            st->flag = 1;
        } else {
            st->rho = rz[0];
            st->beta = beta;
        }
    }
    if (status) return;
    const dev::Chunk ch = dev::block_chunk(n, per_block);
    double v[1] = {0.0};
    fcg_rows<L>(n, M, ch, [&](int q) { return pdir_f(z[q], beta, pold[q]); }, [&](int64_t i, double sum) {
        const double pi = pdir_f(z[i], beta, pold[i]);
        pnew[i] = pi;
        w[i] = sum;
        v[0] = fma(pi, sum, v[0]);
    });
    dev::store_partials<TBF, 1>(v, partials + (size_t)S_DELTA * kMaxBlocks, gridDim.x,
                                dev::xcd_block(blockIdx.x, gridDim.x));
}

// x += alpha p, r -= alpha w and the partials of ||r||^2.  Prologue:
// delta = p.w (a breakdown when <= 0) and alpha = rho / delta.
__global__ __launch_bounds__(TBF) void k_fcg_update(int64_t n, double *__restrict__ x, double *__restrict__ r,
                                                    const double *__restrict__ p, const double *__restrict__ w,
                                                    FcgState *st, double *partials, int64_t per_block) {
    if (st->flag) return;
    double d[1];
    dev::reduce_partials<TBF, 1>(partials + (size_t)S_DELTA * kMaxBlocks, gridDim.x, d);
    const double delta = d[0];
    const int status = !(delta > 0.0) ? (isfinite(delta) ? APCG_SOLVE_BREAKDOWN_PAP : APCG_SOLVE_NAN) : 0;
    const double alpha = status ? 0.0 : st->rho / delta;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        st->delta = delta;
        if (status) {
            st->status = status;
            st->flag = 1;
        } else {
            st->alpha = alpha;
        }
    }
    if (status) return;
    const dev::Chunk ch = dev::block_chunk(n, per_block);
    double v[1] = {0.0};
    for (int64_t i = ch.lo + threadIdx.x; i < ch.hi; i += TBF) {
        x[i] = fma(alpha, p[i], x[i]);
        const double ri = fma(-alpha, w[i], r[i]);
        r[i] = ri;
        v[0] = fma(ri, ri, v[0]);
    }
    dev::store_partials<TBF, 1>(v, partials + (size_t)S_RES * kMaxBlocks, gridDim.x,
                                dev::xcd_block(blockIdx.x, gridDim.x));
}

// Writes the result record; with a fallback solve, adds its iterations.
// After the flexible phase: gate[0] = 1 when it ended in a breakdown, a
// rejected polynomial or a stall (not a setup error) and the fallback is
// enabled, gate[1] = the iterations left for the Jacobi-PCG fallback.  The
// fallback solve queued after it reads the gate on the device, so the host
// never waits for this decision.
__global__ void k_fcg_gate(const FcgState *st, int32_t *gate, int32_t maxit, int fallback) {
    if (threadIdx.x != 0) return;
    const int bad = APCG_SOLVE_BREAKDOWN_PAP | APCG_SOLVE_BREAKDOWN_RZ | APCG_SOLVE_STALL;
    const int32_t done = max(st->rec[0].its, st->rec[1].its);
    gate[0] = fallback && (st->status & bad) && !(st->status & APCG_SOLVE_SETUP_ERROR) ? 1 : 0;
    gate[1] = max(0, maxit - done);
}

__global__ void k_fcg_finish(const FcgState *st, const apcg_solve_info *fallback, const int32_t *gate,
                             apcg_solve_info *out) {
    if (threadIdx.x != 0) return;
    int status = st->status ? st->status : APCG_SOLVE_MAXIT;
    const FcgRec last = st->rec[0].its >= st->rec[1].its ? st->rec[0] : st->rec[1];
    apcg_solve_info o;
    o.fcg_iterations = last.its;
    o.half_steps = 0;
    o.ref_norm = st->ref;
    if (fallback && gate[0]) {
        o.iterations = last.its + fallback->iterations;
        o.status = fallback->status | APCG_SOLVE_FALLBACK | status;
        o.res_norm = fallback->res_norm;
    } else {
        o.iterations = last.its;
        o.status = status;
        o.res_norm = last.res;
    }
    *out = o;
}

struct FcgCache {
    int device = 0;
    int64_t cap = 0;
    double *ws = nullptr;       // 9 * cap: r, dinv, z, p0, p1, w, t0, t1, t2
    FcgState *st = nullptr;
    apcg_info fb_info = nullptr;  // fallback solve record
    int32_t *pinned = nullptr;    // flag, status pairs
    EventRef poll_ev[kMaxLookahead];
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    const void *gkey[10] = {};
    int32_t gK = 0;
};

}  // namespace

static std::mutex g_fcg_mu;
static std::vector<std::pair<uint64_t, FcgCache *>> g_fcg;

static FcgCache *fcg_cache(apcg_ctx c) {
    std::lock_guard<std::mutex> lk(g_fcg_mu);
    for (auto &p : g_fcg)
        if (p.first == c->id) return p.second;
    FcgCache *s = new FcgCache();
    s->device = c->device;
    g_fcg.emplace_back(c->id, s);
    return s;
}

void fcg_cache_release(uint64_t ctx_id, int device) {
    FcgCache *s = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_fcg_mu);
        for (auto it = g_fcg.begin(); it != g_fcg.end(); ++it)
            if (it->first == ctx_id) {
                s = it->second;
                g_fcg.erase(it);
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
    if (s->fb_info) apcg_info_destroy(s->fb_info);
    delete s;
}

}  // namespace apcg

using namespace apcg;

extern "C" apcg_status apcg_fcg_opts_default(apcg_fcg_opts *o) {
    if (!o) return set_error(APCG_ERR_INVALID_ARG, "opts is NULL");
    memset(o, 0, sizeof *o);
    o->stall_min = 50;
    o->stall_frac = 0.1;
    o->fallback = 1;
    return APCG_SUCCESS;
}

extern "C" apcg_status apcg_ksp_solve_fcg_poly(apcg_ctx ctx, apcg_mat A, apcg_vec b, apcg_vec x, double rtol,
                                               int32_t maxit, const float *dev_coeffs, const double *dev_lmax,
                                               const apcg_solve_opts *opts_in, const apcg_fcg_opts *fopts_in,
                                               apcg_info info, int32_t info_index) {
    try {
        if (!ctx || !A || !b || !x || !info || !dev_coeffs || !dev_lmax)
            return set_error(APCG_ERR_INVALID_ARG, "NULL argument");
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
        apcg_fcg_opts fo;
        if (fopts_in) fo = *fopts_in;
        else apcg_fcg_opts_default(&fo);
        if (fo.stall_min < 1 || !(fo.stall_frac >= 0.0)) return set_error(APCG_ERR_INVALID_ARG, "bad stall window");
        int K = std::max(2, opts.iters_per_graph);
        if (K & 1) ++K;
        const int L = std::max(1, std::min(kMaxLookahead, opts.lookahead));

        FcgCache *fc = fcg_cache(ctx);
        const int dev = ctx->device;
        hipStream_t st = ctx->stream;
        Acc acc[4] = {{&x->rec, ACC_RW}, {&info->rec, ACC_W}, {&A->rec, ACC_R}, {&b->rec, ACC_R}};
        apcg_status s;
        if ((s = op_begin(ctx, acc, 4))) return s;
        const int64_t n = A->n;
        if (fc->cap < n || !fc->ws) {
            if (fc->ws) {
                EventRef ev = event_get(dev);
                if (!ev) return set_error(APCG_ERR_HIP, "event creation failed");
                APCG_HIP(hipEventRecord(ev->e, st));
                double *old = fc->ws;
                hipGraphExec_t oe = fc->exec;
                hipGraph_t og = fc->graph;
                defer_release({ev}, [old, oe, og, dev]() {
                    hipSetDevice(dev);
                    if (oe) hipGraphExecDestroy(oe);
                    if (og) hipGraphDestroy(og);
                    hipFree(old);
                });
                fc->exec = nullptr;
                fc->graph = nullptr;
            }
            const int64_t cap = std::max<int64_t>(64, ((n + 63) / 64) * 64);
            APCG_HIP(hipMalloc((void **)&fc->ws, sizeof(double) * 9 * cap));
            fc->cap = cap;
        }
        if (!fc->st) {
            APCG_HIP(hipMalloc((void **)&fc->st, 512));
            APCG_HIP(hipHostMalloc((void **)&fc->pinned, sizeof(int32_t) * 2 * kMaxLookahead, hipHostMallocDefault));
            if ((s = apcg_info_create(dev, 1, &fc->fb_info))) return s;
        }
        const int64_t cap = fc->cap;
        double *r = fc->ws, *dinv = fc->ws + cap, *z = fc->ws + 2 * cap, *pb[2] = {fc->ws + 3 * cap, fc->ws + 4 * cap};
        double *w = fc->ws + 5 * cap, *t[3] = {fc->ws + 6 * cap, fc->ws + 7 * cap, fc->ws + 8 * cap};
        double *part = ctx->partials;  // slices S_INIT, S_DELTA, S_RES, S_RZ
        int G;
        int64_t pbk;
        fcg_grid(n, &G, &pbk);
        const int x0z = opts.x0_is_zero ? 1 : 0;
        // products on the sliced-diagonal copy whenever the pattern allows it
        // (a one-time host analysis per matrix; bitwise the CSR sums)
        int lw = 0;
        if ((s = sdia_analyse(A))) return s;
        if (A->sdia_state == 1) {
            if ((s = prepare_sdia(A, st))) return s;
            lw = sdia_walk(A);
        }
        const dev::RowMat M{A->rowptr, A->col, A->val, A->sdia_off, A->sdia_msk, A->sdia_val, A->sdia_u};
        auto fcheb = lw == 5 ? k_cheb<5> : lw == 7 ? k_cheb<7> : lw == 8 ? k_cheb<8> : lw == 16 ? k_cheb<16>
                   : lw == 32 ? k_cheb<32> : k_cheb<0>;
        auto fprod = lw == 5 ? k_fcg_product<5> : lw == 7 ? k_fcg_product<7> : lw == 8 ? k_fcg_product<8>
                   : lw == 16 ? k_fcg_product<16> : lw == 32 ? k_fcg_product<32> : k_fcg_product<0>;

        hipLaunchKernelGGL(k_fcg_init, dim3(G), dim3(TBF), 0, st, A->n, A->rowptr, A->col, A->val, b->d, x->d, r, dinv,
                           pb[0], part + (size_t)S_INIT * kMaxBlocks, pbk, x0z);
        APCG_CHECK_LAUNCH("k_fcg_init");
        hipLaunchKernelGGL(k_fcg_init_final, dim3(1), dim3(64), 0, st, fc->st,
                           (const double *)(part + (size_t)S_INIT * kMaxBlocks), G, dev_coeffs, dev_lmax, rtol, maxit,
                           fo.stall_min, fo.stall_frac);
        APCG_CHECK_LAUNCH("k_fcg_init_final");
        if (!x0z) {
            hipLaunchKernelGGL(k_fcg_zero_x_if, dim3(G), dim3(TBF), 0, st, x->d, n, pbk, (const FcgState *)fc->st);
            APCG_CHECK_LAUNCH("k_fcg_zero_x_if");
        }
        // z = P r: b_7 -> t[7%3], ..., b_1 -> t[1%3], z.  check: the first
        // step runs the test of the iteration (parity) that just updated r.
        auto precondition = [&](int check, int parity) -> apcg_status {
            for (int j = DEG - 1; j >= 0; --j) {
                const int stage = j == DEG - 1 ? 0 : (j == 0 ? 2 : 1);
                const double *bj1 = stage == 0 ? nullptr : t[(j + 1) % 3];
                const double *bj2 = (stage == 0 || j + 2 == DEG) ? nullptr : t[(j + 2) % 3];
                double *outp = stage == 2 ? z : t[j % 3];
                hipLaunchKernelGGL(fcheb, dim3(G), dim3(TBF), 0, st, A->n, M,
                                   (const double *)r, (const double *)dinv, bj1, bj2, outp, (const double *)w,
                                   fc->st, j, stage, stage == 0 ? check : 0, parity, part, pbk);
                APCG_CHECK_LAUNCH("k_cheb");
            }
            return APCG_SUCCESS;
        };
        // the first application (z0); its r.z is checked by the first product
        if ((s = precondition(0, 0))) return s;

        // iteration k (parity k & 1; K is even, so the parity of the k-th
        // iteration of a captured period is that of the global iteration)
        auto iteration = [&](int k) -> apcg_status {
            const double *pold = pb[(k + 1) & 1];
            double *pnew = pb[k & 1];
            hipLaunchKernelGGL(fprod, dim3(G), dim3(TBF), 0, st, A->n, M, (const double *)z, pold, pnew, w, fc->st,
                               k & 1, part, pbk);
            APCG_CHECK_LAUNCH("k_fcg_product");
            hipLaunchKernelGGL(k_fcg_update, dim3(G), dim3(TBF), 0, st, n, x->d, r, (const double *)pnew,
                               (const double *)w, fc->st, part, pbk);
            APCG_CHECK_LAUNCH("k_fcg_update");
            return precondition(1, k & 1);
        };

        if (maxit > 0) {
            if (opts.mode == APCG_MODE_GRAPH) {
                const void *key[10] = {(const void *)(uintptr_t)A->uid, A->rowptr, A->col, A->val, x->d, fc->ws,
                                       (const void *)ctx->partials, (const void *)(intptr_t)n,
                                       (const void *)(intptr_t)lw, A->sdia_val};
                if (!fc->exec || fc->gK != K || memcmp(key, fc->gkey, sizeof key) != 0) {
                    if (fc->exec) {
                        EventRef ev = event_get(dev);
                        if (ev) hipEventRecord(ev->e, st);
                        hipGraphExec_t oe = fc->exec;
                        hipGraph_t og = fc->graph;
                        defer_release({ev}, [oe, og, dev]() {
                            hipSetDevice(dev);
                            hipGraphExecDestroy(oe);
                            hipGraphDestroy(og);
                        });
                        fc->exec = nullptr;
                        fc->graph = nullptr;
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
                    if (e != hipSuccess) return hip_error(e, "hipStreamEndCapture(fcg)");
                    g_counters.kernel_launches -= (int64_t)(2 + DEG) * K;
                    e = hipGraphInstantiate(&fc->exec, g, nullptr, nullptr, 0);
                    if (e != hipSuccess) {
                        hipGraphDestroy(g);
                        return hip_error(e, "hipGraphInstantiate(fcg)");
                    }
                    fc->graph = g;
                    memcpy(fc->gkey, key, sizeof key);
                    fc->gK = K;
                }
            }
            const int64_t periods = ((int64_t)maxit + K - 1) / K;
            for (int64_t g = 0; g < periods; ++g) {
                if (opts.mode == APCG_MODE_GRAPH) {
                    g_counters.graph_launches++;
                    APCG_HIP(hipGraphLaunch(fc->exec, st));
                } else {
                    for (int j = 1; j <= K; ++j)
                        if ((s = iteration(j))) return s;
                }
                const int slot = (int)(g % L);
                if (!fc->poll_ev[slot]) {
                    fc->poll_ev[slot] = event_get(dev);
                    if (!fc->poll_ev[slot]) return set_error(APCG_ERR_HIP, "event creation failed");
                }
                g_counters.d2h_copies++;
                APCG_HIP(hipMemcpyAsync(&fc->pinned[2 * slot], &fc->st->status, 2 * sizeof(int32_t),
                                        hipMemcpyDeviceToHost, st));
                APCG_HIP(hipEventRecord(fc->poll_ev[slot]->e, st));
                if (g >= L - 1) {
                    const int ps = (int)((g - (L - 1)) % L);
                    g_counters.host_polls++;
                    APCG_HIP(hipEventSynchronize(fc->poll_ev[ps]->e));
                    if (fc->pinned[2 * ps + 1]) break;  // flag
                }
            }
        }
        // Fallback: when the flexible phase ended in a breakdown, a rejected
        // polynomial or a stall, Jacobi-PCG continues from the current x for
        // the iterations left.  The decision is taken on the device: the
        // gate kernel writes it, and the fallback solve, always queued (one
        // graph period ahead of its poll), reads it in its first kernels and
        // is a no-op when not needed -- the host never waits for the
        // flexible phase's outcome.
        int32_t *gate = reinterpret_cast<int32_t *>(reinterpret_cast<char *>(fc->st) + kGateOffset);
        hipLaunchKernelGGL(k_fcg_gate, dim3(1), dim3(64), 0, st, (const FcgState *)fc->st, gate, maxit,
                           fo.fallback ? 1 : 0);
        APCG_CHECK_LAUNCH("k_fcg_gate");
        const apcg_solve_info *fb = nullptr;
        if (fo.fallback) {
            apcg_solve_opts po;
            apcg_solve_opts_default(&po);
            po.mode = opts.mode == APCG_MODE_STREAM || opts.mode == APCG_MODE_HOST_CHECK ? opts.mode : APCG_MODE_GRAPH;
            po.iters_per_graph = opts.iters_per_graph;
            po.lookahead = 1;
            po.x0_is_zero = 0;
            if ((s = pcg_solve_marked(ctx, A, b, x, rtol, maxit, &po, fc->fb_info, 0, nullptr, 0, gate))) return s;
            fb = fc->fb_info->d;
        }
        hipLaunchKernelGGL(k_fcg_finish, dim3(1), dim3(64), 0, st, (const FcgState *)fc->st, fb,
                           (const int32_t *)gate, info->d + info_index);
        APCG_CHECK_LAUNCH("k_fcg_finish");
        return op_end(ctx, acc, 4);
    } catch (const std::bad_alloc &) {
        return set_error(APCG_ERR_OUT_OF_MEMORY, "host allocation failed");
    }
}
