// pcg.hip -- the preconditioned conjugate-gradient hot path with every
// scalar on the device (the PCG loop of Section 3.3 with Jacobi
// preconditioning as in Section 4.1).
//
// One iteration is two kernels, each ending in a deterministic two-stage
// reduction whose last workgroup evaluates the scalar step on the device:
//
//   product:  p_new = D^-1 r + beta p_old  (formed while gathering, so the
//             direction update costs no extra pass), w = A p_new,
//             delta = p_new . w;  epilogue: alpha = rho / delta, or
//             BREAKDOWN_PAP when delta is not positive.
//   update:   x += alpha p_new, r -= alpha w, z = D^-1 r (not stored),
//             rho' = z . r and nu = ||r||^2 (or ||z||^2); epilogue: count
//             the iteration, convergence / NaN / breakdown / iteration-limit
//             tests, beta = rho' / rho.
//
// A device word `flag` is raised on any terminal state; every kernel returns
// immediately when it is set, so work enqueued past convergence is a no-op
// and x is exactly the iterate at convergence.  This is the device-side
// convergence check the paper proposes in Section 5.  p is double-buffered:
// iteration k reads p[(k+1)%2] and writes p[k%2].
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>

#include "internal.h"

namespace apcg {

struct SolveState {
    double rho, delta, alpha, beta;
    double res, ref, rtol, unused;
    int32_t its, maxit, status, flag;
    int32_t zero_x, pad0, pad1, pad2;
};
static_assert(sizeof(SolveState) <= 256, "solve state exceeds its allocation");

namespace {

constexpr int VB = 256;  // block size of the vector-shaped kernels

// The direction entry p_j = z_j + beta p_j with z_j = d_j r_j; written once
// so the stored p and the gathered p agree bit for bit.
__device__ __forceinline__ double pdir(double d, double r, double beta, double pold) {
    return fma(beta, pold, d * r);
}

// ----------------------------------------------------------------- setup
// dinv = 1/diag(A) (or 1), r0 = b - A x0 (or b), p_old = 0 and the initial
// reductions rho0 = z0.r0, reference norm^2, residual norm^2, bad rows.
__global__ __launch_bounds__(VB) void k_pcg_init(int32_t n, const int32_t *__restrict__ rowptr,
                                                 const int32_t *__restrict__ col, const double *__restrict__ val,
                                                 const double *__restrict__ b, double *__restrict__ x,
                                                 double *__restrict__ r, double *__restrict__ dinv,
                                                 double *__restrict__ pold, SolveState *st, double *partials,
                                                 unsigned *counter, int64_t per_block, int x0_zero, int pc,
                                                 int norm_pre, double rtol, int32_t maxit) {
    const dev::Chunk c = dev::block_chunk(n, per_block);
    double rz = 0.0, nref = 0.0, nres = 0.0, bad = 0.0;
    for (int64_t i = c.lo + threadIdx.x; i < c.hi; i += VB) {
        const int s = rowptr[i], e = rowptr[i + 1];
        double diag = 0.0, ax = 0.0;
        bool found = false;
        for (int k = s; k < e; ++k) {
            const int j = col[k];
            const double a = val[k];
            if (j == (int)i) {
                diag = a;
                found = true;
            }
            if (!x0_zero) ax = fma(a, x[j], ax);
        }
        double di = 1.0;
        if (pc == APCG_PC_JACOBI) {
            const bool ok = found && diag > 0.0;
            bad += ok ? 0.0 : 1.0;
            di = ok ? 1.0 / diag : 0.0;
        }
        const double bi = b[i];
        const double ri = x0_zero ? bi : bi - ax;
        r[i] = ri;
        dinv[i] = di;
        pold[i] = 0.0;
        const double zi = di * ri;
        rz = fma(zi, ri, rz);
        if (norm_pre) {
            const double zb = di * bi;
            nref = fma(zb, zb, nref);
            nres = fma(zi, zi, nres);
        } else {
            nref = fma(bi, bi, nref);
            nres = fma(ri, ri, nres);
        }
    }
    if (x0_zero) {
        // x0 is taken as zero (never read above) and written as zero here
        for (int64_t i = c.lo + threadIdx.x; i < c.hi; i += VB) x[i] = 0.0;
    }
    double v[4] = {rz, nref, nres, bad};
    const int lb = dev::xcd_block(blockIdx.x, gridDim.x);
    if (dev::reduce_last_block<VB, 4>(v, partials, gridDim.x, lb, counter) && threadIdx.x == 0) {
        const double rho = v[0], ref = sqrt(v[1]), res = sqrt(v[2]);
        int status = 0, zero_x = 0;
        if (v[3] > 0.0) status = APCG_SOLVE_SETUP_ERROR;
        else if (ref == 0.0) {
            status = APCG_SOLVE_CONVERGED;  // b = 0: the solution is x = 0
            zero_x = 1;
        } else if (!isfinite(res) || !isfinite(ref)) status = APCG_SOLVE_NAN;
        else if (res <= rtol * ref) status = APCG_SOLVE_CONVERGED;
        else if (!(rho > 0.0)) status = isfinite(rho) ? APCG_SOLVE_BREAKDOWN_RZ : APCG_SOLVE_NAN;
        st->rho = rho;
        st->delta = 0.0;
        st->alpha = 0.0;
        st->beta = 0.0;
        st->res = zero_x ? 0.0 : res;
        st->ref = ref;
        st->rtol = rtol;
        st->its = 0;
        st->maxit = maxit;
        st->status = status;
        st->flag = status != 0;
        st->zero_x = zero_x;
    }
}

// x0 was given and b turned out to be zero: x = 0.
__global__ __launch_bounds__(VB) void k_pcg_zero_x_if(double *__restrict__ x, int64_t n, int64_t per_block,
                                                      const SolveState *st) {
    if (!st->zero_x) return;
    const dev::Chunk c = dev::block_chunk(n, per_block);
    for (int64_t i = c.lo + threadIdx.x; i < c.hi; i += VB) x[i] = 0.0;
}

// ----------------------------------------------------------------- product
template <int LPR, int TB>
__global__ __launch_bounds__(TB) void k_pcg_product(int32_t n, const int32_t *__restrict__ rowptr,
                                                    const int32_t *__restrict__ col, const double *__restrict__ val,
                                                    const double *__restrict__ dinv, const double *__restrict__ r,
                                                    const double *__restrict__ pold, double *__restrict__ pnew,
                                                    double *__restrict__ w, SolveState *st, double *partials,
                                                    unsigned *counter, int32_t rows_per_block, int respect_flag) {
    if (respect_flag && st->flag) return;
    const double beta = st->beta;
    constexpr int RPP = TB / LPR;
    const int lb = dev::xcd_block(blockIdx.x, gridDim.x);
    const int row0 = lb * rows_per_block;
    const int row1 = min(n, row0 + rows_per_block);
    const int lane = threadIdx.x % LPR, grp = threadIdx.x / LPR;
    double acc = 0.0;
    for (int base = row0; base < row1; base += RPP) {
        const int row = base + grp;
        double sum = 0.0;
        if (row < row1) {
            const int e = rowptr[row + 1];
            for (int k = rowptr[row] + lane; k < e; k += LPR) {
                const int j = col[k];
                sum = fma(val[k], pdir(dinv[j], r[j], beta, pold[j]), sum);
            }
        }
#pragma unroll
        for (int o = LPR / 2; o > 0; o >>= 1) sum += __shfl_xor(sum, o, LPR);
        if (row < row1 && lane == 0) {
            const double pi = pdir(dinv[row], r[row], beta, pold[row]);
            pnew[row] = pi;
            w[row] = sum;
            acc = fma(pi, sum, acc);
        }
    }
    double v[1] = {acc};
    if (dev::reduce_last_block<TB, 1>(v, partials, gridDim.x, lb, counter) && threadIdx.x == 0) {
        const double delta = v[0];
        st->delta = delta;
        if (!(delta > 0.0)) {
            st->status |= isfinite(delta) ? APCG_SOLVE_BREAKDOWN_PAP : APCG_SOLVE_NAN;
            st->flag = 1;
        } else {
            st->alpha = st->rho / delta;
        }
    }
}

// ----------------------------------------------------------------- update
__global__ __launch_bounds__(VB) void k_pcg_update(int64_t n, double *__restrict__ x, double *__restrict__ r,
                                                   const double *__restrict__ p, const double *__restrict__ w,
                                                   const double *__restrict__ dinv, SolveState *st,
                                                   double *partials, unsigned *counter, int64_t per_block,
                                                   int norm_pre) {
    if (st->flag) return;
    const double alpha = st->alpha;
    const dev::Chunk c = dev::block_chunk(n, per_block);
    double rz = 0.0, nn = 0.0;
    for (int64_t i = c.lo + threadIdx.x; i < c.hi; i += VB) {
        const double xi = fma(alpha, p[i], x[i]);
        const double ri = fma(-alpha, w[i], r[i]);
        x[i] = xi;
        r[i] = ri;
        const double zi = dinv[i] * ri;
        rz = fma(zi, ri, rz);
        nn = norm_pre ? fma(zi, zi, nn) : fma(ri, ri, nn);
    }
    double v[2] = {rz, nn};
    const int lb = dev::xcd_block(blockIdx.x, gridDim.x);
    if (dev::reduce_last_block<VB, 2>(v, partials, gridDim.x, lb, counter) && threadIdx.x == 0) {
        const double rho_new = v[0];
        const double res = sqrt(v[1]);
        const int its = st->its + 1;
        st->its = its;
        st->res = res;
        int status = 0;
        if (!isfinite(res) || !isfinite(rho_new)) status = APCG_SOLVE_NAN;
        else if (res <= st->rtol * st->ref) status = APCG_SOLVE_CONVERGED;
        else if (!(rho_new > 0.0)) status = APCG_SOLVE_BREAKDOWN_RZ;
        else if (its >= st->maxit) status = APCG_SOLVE_MAXIT;
        if (status) {
            st->status |= status;
            st->flag = 1;
        } else {
            st->beta = rho_new / st->rho;
            st->rho = rho_new;
        }
    }
}

// Copies the terminal state into the caller's info record.
__global__ void k_pcg_finish(SolveState *st, apcg_solve_info *out) {
    if (threadIdx.x != 0) return;
    int status = st->status;
    if (status == 0) status = APCG_SOLVE_MAXIT;  // maxit reached before any test fired
    out->iterations = st->its;
    out->status = status;
    out->fcg_iterations = 0;
    out->reserved = 0;
    out->res_norm = st->res;
    out->ref_norm = st->ref;
}

__global__ void k_tune_state(SolveState *st) {
    if (threadIdx.x != 0) return;
    st->flag = 0;
    st->beta = 0.5;
    st->rho = 1.0;
    st->status = 0;
}

__global__ __launch_bounds__(VB) void k_tune_fill(double *r, double *dinv, double *p, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * VB + threadIdx.x; i < n; i += (int64_t)gridDim.x * VB) {
        r[i] = 1.0 + 1e-3 * (double)(i % 97);
        dinv[i] = 0.25;
        p[i] = 0.125;
    }
}

using ProductFn = void (*)(int32_t, const int32_t *, const int32_t *, const double *, const double *,
                           const double *, const double *, double *, double *, SolveState *, double *, unsigned *,
                           int32_t, int);

template <int TB>
ProductFn product_fn_tb(int lpr) {
    switch (lpr) {
        case 1: return k_pcg_product<1, TB>;
        case 2: return k_pcg_product<2, TB>;
        case 4: return k_pcg_product<4, TB>;
        case 8: return k_pcg_product<8, TB>;
        case 16: return k_pcg_product<16, TB>;
        case 32: return k_pcg_product<32, TB>;
        case 64: return k_pcg_product<64, TB>;
        default: return nullptr;
    }
}

ProductFn product_fn(int lpr, int tb) { return tb == 512 ? product_fn_tb<512>(lpr) : product_fn_tb<256>(lpr); }

// Launch geometry of one solve.
struct Plan {
    int32_t n;
    ProductFn prod;
    int tb;
    int g_prod;
    int32_t rpb;
    int g_vec;
    int64_t pb_vec;
};

apcg_status make_plan(const apcg_mat_s *A, const apcg_spmv_config &cfg, Plan *pl) {
    pl->n = A->n;
    pl->tb = cfg.block_size == 512 ? 512 : 256;
    pl->prod = product_fn(cfg.lanes_per_row, pl->tb);
    if (!pl->prod) return set_error(APCG_ERR_INVALID_ARG, "unsupported lanes_per_row");
    const int64_t rpp = pl->tb / cfg.lanes_per_row;
    pl->g_prod = normalise_blocks(cfg.blocks, (A->n + rpp - 1) / rpp);
    int64_t rpb = ((int64_t)A->n + pl->g_prod - 1) / pl->g_prod;
    pl->rpb = (int32_t)std::max<int64_t>(1, rpb);
    elementwise_grid(A->n, &pl->g_vec, &pl->pb_vec);
    return APCG_SUCCESS;
}

struct Bufs {
    const apcg_mat_s *A;
    double *x;
    const double *b;
    Workspace ws;
    double *partials;
    unsigned *counters;
};

apcg_status launch_product(hipStream_t s, const Plan &pl, const Bufs &bf, int iter, int respect_flag = 1) {
    const double *pold = bf.ws.p((iter + 1) & 1);
    double *pnew = bf.ws.p(iter & 1);
    hipLaunchKernelGGL(pl.prod, dim3(pl.g_prod), dim3(pl.tb), 0, s, pl.n, bf.A->rowptr, bf.A->col, bf.A->val,
                       (const double *)bf.ws.dinv(), (const double *)bf.ws.r(), pold, pnew, bf.ws.w(), bf.ws.state,
                       bf.partials, bf.counters + CNT_PCG_PRODUCT, pl.rpb, respect_flag);
    APCG_CHECK_LAUNCH("k_pcg_product");
    return APCG_SUCCESS;
}

apcg_status launch_update(hipStream_t s, const Plan &pl, const Bufs &bf, int iter, int norm_pre) {
    const double *p = bf.ws.p(iter & 1);
    hipLaunchKernelGGL(k_pcg_update, dim3(pl.g_vec), dim3(VB), 0, s, (int64_t)pl.n, bf.x, bf.ws.r(), p,
                       (const double *)bf.ws.w(), (const double *)bf.ws.dinv(), bf.ws.state, bf.partials,
                       bf.counters + CNT_PCG_UPDATE, pl.pb_vec, norm_pre);
    APCG_CHECK_LAUNCH("k_pcg_update");
    return APCG_SUCCESS;
}

apcg_status get_graph(apcg_ctx c, const Plan &pl, const Bufs &bf, int K, int pc, int norm_pre,
                      hipGraphExec_t *exec) {
    GraphKey key{bf.A, bf.x, bf.ws.base, K, bf.A->cfg.lanes_per_row, pl.tb, pl.g_prod, pc, norm_pre};
    for (auto &g : c->graphs)
        if (g.key == key) {
            *exec = g.exec;
            return APCG_SUCCESS;
        }
    hipGraph_t graph = nullptr;
    APCG_HIP(hipStreamBeginCapture(c->stream, hipStreamCaptureModeRelaxed));
    apcg_status st = APCG_SUCCESS;
    for (int j = 1; j <= K && st == APCG_SUCCESS; ++j) {
        st = launch_product(c->stream, pl, bf, j);
        if (st == APCG_SUCCESS) st = launch_update(c->stream, pl, bf, j, norm_pre);
    }
    hipError_t e = hipStreamEndCapture(c->stream, &graph);
    if (st != APCG_SUCCESS) {
        if (graph) hipGraphDestroy(graph);
        return st;
    }
    if (e != hipSuccess) return hip_error(e, "hipStreamEndCapture");
    g_counters.kernel_launches -= 2 * K;  // captured, not launched
    hipGraphExec_t ex = nullptr;
    e = hipGraphInstantiate(&ex, graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        hipGraphDestroy(graph);
        return hip_error(e, "hipGraphInstantiate");
    }
    if (c->graphs.size() >= 4) {
        GraphEntry old = c->graphs.front();
        c->graphs.erase(c->graphs.begin());
        EventRef ev = event_get(c->device);
        if (ev) hipEventRecord(ev->e, c->stream);
        int dev = c->device;
        defer_release({ev}, [old, dev]() {
            hipSetDevice(dev);
            hipGraphExecDestroy(old.exec);
            hipGraphDestroy(old.graph);
        });
    }
    c->graphs.push_back({key, ex, graph});
    *exec = ex;
    return APCG_SUCCESS;
}

// Queues one poll point: copy the device flag to pinned slot `slot` and
// record an event behind it.
apcg_status queue_poll(apcg_ctx c, const Bufs &bf, int slot) {
    if (!c->poll_ev[slot]) {
        c->poll_ev[slot] = event_get(c->device);
        if (!c->poll_ev[slot]) return set_error(APCG_ERR_HIP, "event creation failed");
    }
    g_counters.d2h_copies++;
    APCG_HIP(hipMemcpyAsync(&c->pinned_flags[slot], &bf.ws.state->flag, sizeof(int32_t), hipMemcpyDeviceToHost,
                            c->stream));
    APCG_HIP(hipEventRecord(c->poll_ev[slot]->e, c->stream));
    return APCG_SUCCESS;
}

// Waits for poll point `slot` (queued `lookahead` periods ago) and reports
// whether the device had already stopped.
apcg_status check_poll(apcg_ctx c, int slot, bool *done) {
    g_counters.host_polls++;
    APCG_HIP(hipEventSynchronize(c->poll_ev[slot]->e));
    *done = c->pinned_flags[slot] != 0;
    return APCG_SUCCESS;
}

apcg_status timed_launch(apcg_ctx c, int kind, int iter, const std::function<apcg_status()> &launch) {
    const int idx = c->tpairs;
    if (idx >= 4096) return launch();
    if ((int)c->tev.size() < 2 * (idx + 1)) {
        for (int k = 0; k < 2; ++k) {
            hipEvent_t e;
            APCG_HIP(hipEventCreate(&e));
            c->tev.push_back(e);
        }
    }
    if ((int)c->tkind.size() < 2 * (idx + 1)) c->tkind.resize(2 * (idx + 1));
    APCG_HIP(hipEventRecord(c->tev[2 * idx], c->stream));
    apcg_status s = launch();
    if (s) return s;
    APCG_HIP(hipEventRecord(c->tev[2 * idx + 1], c->stream));
    c->tkind[2 * idx] = kind;
    c->tkind[2 * idx + 1] = iter;
    c->tpairs = idx + 1;
    return APCG_SUCCESS;
}

}  // namespace
}  // namespace apcg

using namespace apcg;

extern "C" {

apcg_status apcg_solve_opts_default(apcg_solve_opts *opts) {
    if (!opts) return set_error(APCG_ERR_INVALID_ARG, "opts is NULL");
    memset(opts, 0, sizeof *opts);
    opts->pc = APCG_PC_JACOBI;
    opts->norm_type = APCG_NORM_UNPRECONDITIONED;
    opts->mode = APCG_MODE_GRAPH;
    opts->iters_per_graph = 16;
    opts->lookahead = 2;
    opts->x0_is_zero = 0;
    opts->kernel_timing = 0;
    return APCG_SUCCESS;
}

apcg_status apcg_ksp_solve(apcg_ctx ctx, apcg_mat A, apcg_vec b, apcg_vec x, double rtol, int32_t maxit,
                           const apcg_solve_opts *opts_in, apcg_info info, int32_t info_index) {
    try {
        if (!A || !b || !x || !info) return set_error(APCG_ERR_INVALID_ARG, "NULL argument");
        if (b->n != A->n || x->n != A->n) return set_error(APCG_ERR_INVALID_ARG, "dimension mismatch");
        if (b == x || (b->d == x->d && A->n > 0)) return set_error(APCG_ERR_INVALID_ARG, "b and x must not alias");
        if (b->device != A->device || x->device != A->device || info->device != A->device)
            return set_error(APCG_ERR_INVALID_ARG, "operands on different devices");
        if (info_index < 0 || info_index >= info->count)
            return set_error(APCG_ERR_INVALID_ARG, "info index out of range");
        if (!(rtol >= 0.0) || !std::isfinite(rtol)) return set_error(APCG_ERR_INVALID_ARG, "rtol must be finite and >= 0");
        if (maxit < 0) return set_error(APCG_ERR_INVALID_ARG, "maxit must be >= 0");
        apcg_solve_opts opts;
        if (opts_in) opts = *opts_in;
        else apcg_solve_opts_default(&opts);
        if (opts.pc != APCG_PC_NONE && opts.pc != APCG_PC_JACOBI)
            return set_error(APCG_ERR_UNSUPPORTED, "unsupported preconditioner for apcg_ksp_solve");
        if (opts.norm_type != APCG_NORM_UNPRECONDITIONED && opts.norm_type != APCG_NORM_PRECONDITIONED)
            return set_error(APCG_ERR_INVALID_ARG, "unknown norm type");
        if (opts.mode < APCG_MODE_GRAPH || opts.mode > APCG_MODE_HOST_CHECK)
            return set_error(APCG_ERR_INVALID_ARG, "unknown mode");
        if (opts.iters_per_graph < 1) return set_error(APCG_ERR_INVALID_ARG, "iters_per_graph must be >= 1");
        if (opts.lookahead < 1 || opts.lookahead > kMaxLookahead)
            return set_error(APCG_ERR_INVALID_ARG, "lookahead must be in [1, 8]");
        int K = opts.iters_per_graph;
        if (K & 1) ++K;  // even: the direction buffers alternate per iteration
        if (opts.kernel_timing) opts.mode = APCG_MODE_STREAM;

        apcg_ctx c = nullptr;
        apcg_status s = resolve_ctx(ctx, A->device, &c);
        if (s) return s;
        Acc acc[4] = {{&x->rec, ACC_RW}, {&info->rec, ACC_W}, {&A->rec, ACC_R}, {&b->rec, ACC_R}};
        if ((s = op_begin(c, acc, 4))) return s;
        if ((s = ensure_workspace(c, A->n))) return s;
        Plan pl;
        if ((s = make_plan(A, A->cfg, &pl))) return s;
        Bufs bf{A, x->d, b->d, c->ws, c->partials, c->counters};
        const int norm_pre = opts.norm_type == APCG_NORM_PRECONDITIONED;
        hipStream_t st = c->stream;

        hipLaunchKernelGGL(k_pcg_init, dim3(pl.g_vec), dim3(VB), 0, st, A->n, A->rowptr, A->col, A->val, b->d, x->d,
                           c->ws.r(), c->ws.dinv(), c->ws.p(0), c->ws.state, c->partials,
                           c->counters + CNT_PCG_INIT, pl.pb_vec, opts.x0_is_zero ? 1 : 0, opts.pc, norm_pre, rtol,
                           maxit);
        APCG_CHECK_LAUNCH("k_pcg_init");
        if (!opts.x0_is_zero) {
            hipLaunchKernelGGL(k_pcg_zero_x_if, dim3(pl.g_vec), dim3(VB), 0, st, x->d, (int64_t)A->n, pl.pb_vec,
                               (const SolveState *)c->ws.state);
            APCG_CHECK_LAUNCH("k_pcg_zero_x_if");
        }

        if (opts.kernel_timing) {
            c->tpairs = 0;
        }

        if (maxit > 0) {
            const int L = opts.lookahead;
            if (opts.mode == APCG_MODE_GRAPH) {
                hipGraphExec_t exec = nullptr;
                if ((s = get_graph(c, pl, bf, K, opts.pc, norm_pre, &exec))) return s;
                const int64_t ngraphs = ((int64_t)maxit + K - 1) / K;
                for (int64_t g = 0; g < ngraphs; ++g) {
                    g_counters.graph_launches++;
                    APCG_HIP(hipGraphLaunch(exec, st));
                    if ((s = queue_poll(c, bf, (int)(g % L)))) return s;
                    if (g >= L - 1) {
                        bool done = false;
                        if ((s = check_poll(c, (int)((g - (L - 1)) % L), &done))) return s;
                        if (done) break;
                    }
                }
            } else if (opts.mode == APCG_MODE_STREAM) {
                int64_t period = 0;
                for (int32_t k = 1; k <= maxit; ++k) {
                    if (opts.kernel_timing) {
                        if ((s = timed_launch(c, 0, k, [&]() { return launch_product(st, pl, bf, k); }))) return s;
                        if ((s = timed_launch(c, 1, k, [&]() { return launch_update(st, pl, bf, k, norm_pre); })))
                            return s;
                    } else {
                        if ((s = launch_product(st, pl, bf, k))) return s;
                        if ((s = launch_update(st, pl, bf, k, norm_pre))) return s;
                    }
                    if (k % K == 0 || k == maxit) {
                        if ((s = queue_poll(c, bf, (int)(period % L)))) return s;
                        if (period >= L - 1) {
                            bool done = false;
                            if ((s = check_poll(c, (int)((period - (L - 1)) % L), &done))) return s;
                            if (done) break;
                        }
                        ++period;
                    }
                }
            } else {  // APCG_MODE_HOST_CHECK: the host reads the flag after every kernel
                for (int32_t k = 1; k <= maxit; ++k) {
                    bool done = false;
                    if ((s = launch_product(st, pl, bf, k))) return s;
                    if ((s = queue_poll(c, bf, 0))) return s;
                    g_counters.host_syncs++;
                    if ((s = check_poll(c, 0, &done))) return s;
                    g_counters.host_polls--;
                    if (done) break;
                    if ((s = launch_update(st, pl, bf, k, norm_pre))) return s;
                    if ((s = queue_poll(c, bf, 0))) return s;
                    g_counters.host_syncs++;
                    if ((s = check_poll(c, 0, &done))) return s;
                    g_counters.host_polls--;
                    if (done) break;
                }
            }
        }
        hipLaunchKernelGGL(k_pcg_finish, dim3(1), dim3(64), 0, st, c->ws.state, info->d + info_index);
        APCG_CHECK_LAUNCH("k_pcg_finish");
        if (opts.kernel_timing) {
            c->tdone = event_get(c->device);
            if (c->tdone) APCG_HIP(hipEventRecord(c->tdone->e, st));
        }
        return op_end(c, acc, 4);
    } catch (const std::bad_alloc &) {
        return set_error(APCG_ERR_OUT_OF_MEMORY, "host allocation failed");
    }
}

apcg_status apcg_ctx_kernel_times(apcg_ctx ctx, int32_t kind, double *mean_us, int32_t *count) {
    if (!ctx || !mean_us || !count) return set_error(APCG_ERR_INVALID_ARG, "NULL argument");
    if (kind != 0 && kind != 1) return set_error(APCG_ERR_INVALID_ARG, "kind must be 0 or 1");
    if (!ctx->tdone) return set_error(APCG_ERR_INVALID_STATE, "no timed solve on this context");
    APCG_HIP(hipSetDevice(ctx->device));
    g_counters.host_syncs++;
    APCG_HIP(hipEventSynchronize(ctx->tdone->e));
    // iterations actually performed: launches past convergence returned at once
    SolveState hs;
    g_counters.d2h_copies++;
    APCG_HIP(hipMemcpy(&hs, ctx->ws.state, sizeof hs, hipMemcpyDeviceToHost));
    double total = 0.0;
    int32_t n = 0;
    for (int i = 0; i < ctx->tpairs; ++i) {
        if (ctx->tkind[2 * i] != kind || ctx->tkind[2 * i + 1] > hs.its) continue;
        float ms = 0.f;
        APCG_HIP(hipEventElapsedTime(&ms, ctx->tev[2 * i], ctx->tev[2 * i + 1]));
        total += ms;
        ++n;
    }
    *count = n;
    *mean_us = n ? 1000.0 * total / n : 0.0;
    return APCG_SUCCESS;
}

apcg_status apcg_mat_autotune(apcg_mat A, apcg_ctx ctx, int32_t reps, apcg_spmv_config *best, double *best_us) {
    try {
        if (!A || !ctx || reps < 1) return set_error(APCG_ERR_INVALID_ARG, "bad autotune arguments");
        if (ctx->device != A->device) return set_error(APCG_ERR_INVALID_ARG, "operands on different devices");
        if (ctx->type == APCG_STREAM_GLOBAL_BLOCKING)
            return set_error(APCG_ERR_INVALID_ARG, "autotune needs a default-stream context");
        Acc acc[1] = {{&A->rec, ACC_R}};
        apcg_status s;
        if ((s = op_begin(ctx, acc, 1))) return s;
        if ((s = ensure_workspace(ctx, A->n))) return s;
        hipStream_t st = ctx->stream;
        const int64_t n = A->n;
        hipLaunchKernelGGL(k_tune_fill, dim3(1024), dim3(VB), 0, st, ctx->ws.r(), ctx->ws.dinv(), ctx->ws.p(0), n);
        APCG_CHECK_LAUNCH("k_tune_fill");
        hipLaunchKernelGGL(k_tune_state, dim3(1), dim3(64), 0, st, ctx->ws.state);
        APCG_CHECK_LAUNCH("k_tune_state");
        Bufs bf{A, nullptr, nullptr, ctx->ws, ctx->partials, ctx->counters};
        const double per_row = n > 0 ? (double)A->nnz / n : 1.0;
        hipEvent_t e0, e1;
        APCG_HIP(hipEventCreate(&e0));
        APCG_HIP(hipEventCreate(&e1));
        double best_t = 1e300;
        apcg_spmv_config best_cfg = A->cfg;
        for (int lpr : {1, 2, 4, 8, 16, 32, 64}) {
            if (lpr > 1 && lpr > 4 * std::max(1.0, per_row)) continue;
            for (int tb : {256, 512}) {
                for (int blocks : {1024, 2048, 4096, 8192}) {
                    apcg_spmv_config cfg{lpr, tb, blocks, 0};
                    Plan pl;
                    if ((s = make_plan(A, cfg, &pl))) return s;
                    if (pl.g_prod < blocks && blocks > 1024) continue;  // same grid as a smaller candidate
                    for (int w = 0; w < 2; ++w)
                        if ((s = launch_product(st, pl, bf, 1, 0))) return s;
                    APCG_HIP(hipEventRecord(e0, st));
                    for (int r = 0; r < reps; ++r)
                        if ((s = launch_product(st, pl, bf, 1, 0))) return s;
                    APCG_HIP(hipEventRecord(e1, st));
                    g_counters.host_syncs++;
                    APCG_HIP(hipEventSynchronize(e1));
                    float ms = 0.f;
                    APCG_HIP(hipEventElapsedTime(&ms, e0, e1));
                    const double us = 1000.0 * ms / reps;
                    if (us < best_t) {
                        best_t = us;
                        best_cfg = cfg;
                    }
                }
            }
        }
        hipEventDestroy(e0);
        hipEventDestroy(e1);
        A->cfg = best_cfg;
        if (best) *best = best_cfg;
        if (best_us) *best_us = best_t;
        return op_end(ctx, acc, 1);
    } catch (const std::bad_alloc &) {
        return set_error(APCG_ERR_OUT_OF_MEMORY, "host allocation failed");
    }
}

}  // extern "C"
