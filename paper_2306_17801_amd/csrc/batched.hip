// batched.hip -- many independent Jacobi-PCG solves in one persistent launch.
//
// Each workgroup takes the next system from a device work queue (ordered by
// decreasing estimated cost, so the longest solves start first) and runs the
// whole PCG iteration for it: the same steps, tests and order as the
// single-system path (the PCG loop of Section 3.3), with the two grid-wide
// reductions per iteration replaced by workgroup reductions.  Nothing in a
// solve crosses a workgroup, so there is no inter-workgroup synchronisation at
// all; the queue index is the only atomic.  Launched once per batch (captured
// in a hipGraph together with the queue reset), every scalar stays in
// registers/LDS and no iteration involves the host.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <vector>

#include "internal.h"

namespace apcg {

struct BatchSys {
    const int32_t *rowptr;
    const int32_t *col;
    const double *val;
    const double *b;
    double *x;
    double *ws;  // 6 n doubles: r, dinv, p0, p1, w, z
    // the matrix's sliced-diagonal copy (8 offset slots per slice), used by
    // the segmented schedule's product when the matrix's SpMV schedule is
    // APCG_SPMV_SDIA; null otherwise
    const int32_t *soff;
    const uint64_t *smask;
    const double *sval;
    int32_t n;
    int32_t U;
};

// segmented schedule (below)
apcg_status seg_solve(apcg_ctx ctx, int32_t nsys, const BatchSys *hsys, const BatchSys *d_sys, double rtol,
                      int32_t maxit, const apcg_solve_opts &opts, apcg_solve_info *d_info);

namespace {

__device__ __forceinline__ double pdir_b(double d, double r, double beta, double pold) {
    return fma(beta, pold, d * r);
}

// Sum of v over the workgroup, returned to every thread; the same fixed tree
// in every thread, so all threads hold identical totals.
template <int TB, int NV>
__device__ __forceinline__ void block_allreduce(double (&v)[NV], double *lds) {
    constexpr int NW = TB / 64;
#pragma unroll
    for (int k = 0; k < NV; ++k) v[k] = dev::wave_sum(v[k]);
    const int wid = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (lane == 0) {
#pragma unroll
        for (int k = 0; k < NV; ++k) lds[k * NW + wid] = v[k];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        double s = lds[k * NW];
        for (int w = 1; w < NW; ++w) s += lds[k * NW + w];
        v[k] = s;
    }
    __syncthreads();  // lds may be reused right after
}

// Row i of A p with p_j = d_j r_j + beta pold_j formed while gathering; rows
// of up to 8 entries issue every gather before the first multiply-add.  Both
// branches add in column-storage order.
template <class PI, class PD>
__device__ __forceinline__ double row_product(PI col, PD val, int s, int e, int row, PD dinv, PD r, PD pold,
                                              double beta) {
    const int len = e - s;
    double sum = 0.0;
    if (len <= 8) {
        int jj[8];
        double aa[8], pj[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const bool in = q < len;
            jj[q] = in ? col[s + q] : row;
            aa[q] = in ? val[s + q] : 0.0;
        }
#pragma unroll
        for (int q = 0; q < 8; ++q) pj[q] = pdir_b(dinv[jj[q]], r[jj[q]], beta, pold[jj[q]]);
#pragma unroll
        for (int q = 0; q < 8; ++q)
            if (q < len) sum = fma(aa[q], pj[q], sum);
    } else {
        for (int k = s; k < e; ++k) {
            const int j = col[k];
            sum = fma(val[k], pdir_b(dinv[j], r[j], beta, pold[j]), sum);
        }
    }
    return sum;
}

// Row i of A p with p_j = z_j + beta pold_j (z = D^-1 r as stored by the
// segmented schedule; the same rounded value as d_j r_j above, so the sums are
// bitwise those of row_product).
__device__ __forceinline__ double row_product_z(const dev::glob_t<int32_t> *col, const dev::glob_t<double> *val,
                                                int s, int e, int row, const dev::glob_t<double> *z,
                                                const dev::glob_t<double> *pold, double beta) {
    const int len = e - s;
    double sum = 0.0;
    if (len <= 8) {
        int jj[8];
        double aa[8], pj[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const bool in = q < len;
            jj[q] = in ? col[s + q] : row;
            aa[q] = in ? val[s + q] : 0.0;
        }
#pragma unroll
        for (int q = 0; q < 8; ++q) pj[q] = fma(beta, pold[jj[q]], z[jj[q]]);
#pragma unroll
        for (int q = 0; q < 8; ++q)
            if (q < len) sum = fma(aa[q], pj[q], sum);
    } else {
        for (int k = s; k < e; ++k) {
            const int j = col[k];
            sum = fma(val[k], fma(beta, pold[j], z[j]), sum);
        }
    }
    return sum;
}

template <int TB>
__device__ void solve_one(const BatchSys &S, double rtol, int32_t maxit, int x0_zero, int pc, int norm_pre,
                          apcg_solve_info *out, double *lds) {
    const int n = S.n;
    // global pointers: the system's pointers come from a table in memory
    // (generic to the compiler), and flat accesses would also count in lgkmcnt
    auto *r = dev::glb(S.ws), *dinv = dev::glb(S.ws + n), *pbuf0 = dev::glb(S.ws + 2 * (int64_t)n);
    auto *pbuf1 = dev::glb(S.ws + 3 * (int64_t)n), *w = dev::glb(S.ws + 4 * (int64_t)n), *x = dev::glb(S.x);
    const auto *b = dev::glb(S.b), *val = dev::glb(S.val);
    const auto *rowptr = dev::glb(S.rowptr), *col = dev::glb(S.col);

    // setup: dinv, r0, p_old = 0, rho0, reference and residual norms
    double v4[4] = {0.0, 0.0, 0.0, 0.0};  // z.r, residual^2, reference^2, bad diagonals
    for (int i = threadIdx.x; i < n; i += TB) {
        const int s = rowptr[i], e = rowptr[i + 1];
        double diag = 0.0, ax = 0.0;
        bool found = false;
        for (int k = s; k < e; ++k) {
            const int j = col[k];
            const double a = val[k];
            if (j == i) {
                diag = a;
                found = true;
            }
            if (!x0_zero) ax = fma(a, x[j], ax);
        }
        double di = 1.0;
        if (pc == APCG_PC_JACOBI) {
            const bool ok = found && diag > 0.0;
            v4[3] += ok ? 0.0 : 1.0;
            di = ok ? 1.0 / diag : 0.0;
        }
        const double bi = b[i];
        const double ri = x0_zero ? bi : bi - ax;
        r[i] = ri;
        dinv[i] = di;
        pbuf0[i] = 0.0;
        const double zi = di * ri;
        v4[0] = fma(zi, ri, v4[0]);
        if (norm_pre) {
            const double zb = di * bi;
            v4[2] = fma(zb, zb, v4[2]);
            v4[1] = fma(zi, zi, v4[1]);
        } else {
            v4[2] = fma(bi, bi, v4[2]);
            v4[1] = fma(ri, ri, v4[1]);
        }
    }
    // x is written only after every workgroup thread has read x0
    block_allreduce<TB, 4>(v4, lds);
    if (x0_zero)
        for (int i = threadIdx.x; i < n; i += TB) x[i] = 0.0;
    double rho = v4[0];
    double res = sqrt(v4[1]);
    const double ref = sqrt(v4[2]);
    int status = 0, its = 0;
    if (v4[3] > 0.0) status = APCG_SOLVE_SETUP_ERROR;
    else if (ref == 0.0) {
        status = APCG_SOLVE_CONVERGED;
        res = 0.0;
        for (int i = threadIdx.x; i < n; i += TB) x[i] = 0.0;
    } else if (!isfinite(res) || !isfinite(ref)) status = APCG_SOLVE_NAN;
    else if (res <= rtol * ref) status = APCG_SOLVE_CONVERGED;
    else if (!(rho > 0.0)) status = isfinite(rho) ? APCG_SOLVE_BREAKDOWN_RZ : APCG_SOLVE_NAN;
    else if (maxit <= 0) status = APCG_SOLVE_MAXIT;

    double beta = 0.0;
    for (int k = 1; !status; ++k) {
        const auto *pold = (k & 1) ? pbuf0 : pbuf1;
        auto *pnew = (k & 1) ? pbuf1 : pbuf0;
        double d1[1] = {0.0};
        for (int i = threadIdx.x; i < n; i += TB) {
            const double sum = row_product<decltype(col), decltype(pold)>(col, val, rowptr[i], rowptr[i + 1], i,
                                                                          dinv, r, pold, beta);
            const double pi = pdir_b(dinv[i], r[i], beta, pold[i]);
            pnew[i] = pi;
            w[i] = sum;
            d1[0] = fma(pi, sum, d1[0]);
        }
        block_allreduce<TB, 1>(d1, lds);
        const double delta = d1[0];
        if (!(delta > 0.0)) {
            status = isfinite(delta) ? APCG_SOLVE_BREAKDOWN_PAP : APCG_SOLVE_NAN;
            its = k - 1;
            break;
        }
        const double alpha = rho / delta;
        double v2[2] = {0.0, 0.0};
        for (int i = threadIdx.x; i < n; i += TB) {
            const double xi = fma(alpha, pnew[i], x[i]);
            const double ri = fma(-alpha, w[i], r[i]);
            x[i] = xi;
            r[i] = ri;
            const double zi = dinv[i] * ri;
            v2[0] = fma(zi, ri, v2[0]);
            v2[1] = norm_pre ? fma(zi, zi, v2[1]) : fma(ri, ri, v2[1]);
        }
        block_allreduce<TB, 2>(v2, lds);
        const double rho_new = v2[0];
        res = sqrt(v2[1]);
        its = k;
        if (!isfinite(res) || !isfinite(rho_new)) status = APCG_SOLVE_NAN;
        else if (res <= rtol * ref) status = APCG_SOLVE_CONVERGED;
        else if (!(rho_new > 0.0)) status = APCG_SOLVE_BREAKDOWN_RZ;
        else if (k >= maxit) status = APCG_SOLVE_MAXIT;
        if (!status) {
            beta = rho_new / rho;
            rho = rho_new;
        }
    }
    if (threadIdx.x == 0) {
        out->iterations = its;
        out->status = status;
        out->fcg_iterations = 0;
        out->half_steps = 0;
        out->res_norm = res;
        out->ref_norm = ref;
    }
}

template <int TB>
__global__ __launch_bounds__(TB) void k_pcg_batched(const BatchSys *sys, const int32_t *order, int32_t nsys,
                                                    unsigned *queue, double rtol, int32_t maxit, int x0_zero, int pc,
                                                    int norm_pre, apcg_solve_info *info) {
    __shared__ double lds[4 * (TB / 64)];
    __shared__ int s_next;
    for (;;) {
        if (threadIdx.x == 0) s_next = (int)atomicAdd(queue, 1u);
        __syncthreads();
        const int q = s_next;
        __syncthreads();  // every thread has read s_next before it changes
        if (q >= nsys) return;
        const int id = order[q];
        solve_one<TB>(sys[id], rtol, maxit, x0_zero, pc, norm_pre, info + id, lds);
        __syncthreads();
    }
}

__global__ void k_queue_reset(unsigned *queue) {
    if (threadIdx.x == 0) *queue = 0u;
}

using BatchedFn = void (*)(const BatchSys *, const int32_t *, int32_t, unsigned *, double, int32_t, int, int, int,
                           apcg_solve_info *);

BatchedFn batched_fn(int tb) {
    switch (tb) {
        case 256: return k_pcg_batched<256>;
        case 512: return k_pcg_batched<512>;
        case 1024: return k_pcg_batched<1024>;
        default: return nullptr;
    }
}

uint64_t fnv1a(const void *p, size_t n, uint64_t h = 1469598103934665603ull) {
    const unsigned char *c = (const unsigned char *)p;
    for (size_t i = 0; i < n; ++i) {
        h ^= c[i];
        h *= 1099511628211ull;
    }
    return h;
}

}  // namespace

// Per-context batch resources (kept in a side table keyed by context id).
struct BatchCache {
    int device = 0;
    BatchSys *d_sys = nullptr;
    int32_t *d_order = nullptr;
    unsigned *d_queue = nullptr;
    double *d_ws = nullptr;
    int64_t sys_cap = 0, ws_cap = 0;
    uint64_t desc_hash = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    uint64_t graph_hash = 0;
};

static std::mutex g_batch_mu;
static std::vector<std::pair<uint64_t, BatchCache *>> g_batch;

static BatchCache *batch_cache(apcg_ctx c) {
    std::lock_guard<std::mutex> lk(g_batch_mu);
    for (auto &p : g_batch)
        if (p.first == c->id) return p.second;
    BatchCache *bc = new BatchCache();
    bc->device = c->device;
    g_batch.emplace_back(c->id, bc);
    return bc;
}

void batch_cache_release(uint64_t ctx_id, int device) {
    BatchCache *bc = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_batch_mu);
        for (auto it = g_batch.begin(); it != g_batch.end(); ++it)
            if (it->first == ctx_id) {
                bc = it->second;
                g_batch.erase(it);
                break;
            }
    }
    if (!bc) return;
    hipSetDevice(device);
    if (bc->exec) hipGraphExecDestroy(bc->exec);
    if (bc->graph) hipGraphDestroy(bc->graph);
    if (bc->d_sys) hipFree(bc->d_sys);
    if (bc->d_order) hipFree(bc->d_order);
    if (bc->d_queue) hipFree(bc->d_queue);
    if (bc->d_ws) hipFree(bc->d_ws);
    delete bc;
}

}  // namespace apcg

using namespace apcg;

// The ranges [d, d + n) of the solution vectors must not overlap each other,
// any right-hand side or the system's own b (the kernels write x while other
// systems read b): one sweep over all ranges in address order.
static apcg_status check_batch_ranges(int32_t nsys, const apcg_vec *b, const apcg_vec *x) {
    struct Range {
        uintptr_t lo, hi;
        bool written;
    };
    std::vector<Range> rs;
    rs.reserve(2 * (size_t)nsys);
    for (int32_t i = 0; i < nsys; ++i) {
        if (x[i]->n > 0) rs.push_back({(uintptr_t)x[i]->d, (uintptr_t)(x[i]->d + x[i]->n), true});
        if (b[i]->n > 0) rs.push_back({(uintptr_t)b[i]->d, (uintptr_t)(b[i]->d + b[i]->n), false});
    }
    std::sort(rs.begin(), rs.end(), [](const Range &p, const Range &q) { return p.lo < q.lo; });
    uintptr_t end_written = 0, end_any = 0;
    for (const Range &r : rs) {
        if (r.lo < end_written || (r.written && r.lo < end_any))
            return set_error(APCG_ERR_INVALID_ARG,
                             "a solution vector overlaps another solution vector or a right-hand side");
        if (r.written) end_written = std::max(end_written, r.hi);
        end_any = std::max(end_any, r.hi);
    }
    return APCG_SUCCESS;
}

extern "C" apcg_status apcg_ksp_solve_batched(apcg_ctx ctx, int32_t nsys, const apcg_mat *A, const apcg_vec *b,
                                              const apcg_vec *x, double rtol, int32_t maxit,
                                              const apcg_solve_opts *opts_in, apcg_info info) {
    try {
        if (!ctx || nsys < 1 || !A || !b || !x || !info) return set_error(APCG_ERR_INVALID_ARG, "NULL argument");
        if (info->count < nsys) return set_error(APCG_ERR_INVALID_ARG, "info has fewer records than systems");
        if (!(rtol >= 0.0) || !std::isfinite(rtol)) return set_error(APCG_ERR_INVALID_ARG, "rtol must be finite and >= 0");
        if (maxit < 0) return set_error(APCG_ERR_INVALID_ARG, "maxit must be >= 0");
        if (ctx->type == APCG_STREAM_GLOBAL_BLOCKING && ctx->is_default_global)
            return set_error(APCG_ERR_INVALID_ARG, "pass a context created with apcg_ctx_create");
        apcg_solve_opts opts;
        if (opts_in) opts = *opts_in;
        else apcg_solve_opts_default(&opts);
        if (opts.pc != APCG_PC_NONE && opts.pc != APCG_PC_JACOBI)
            return set_error(APCG_ERR_UNSUPPORTED, "unsupported preconditioner for the batched solve");
        if (opts.norm_type != APCG_NORM_UNPRECONDITIONED && opts.norm_type != APCG_NORM_PRECONDITIONED)
            return set_error(APCG_ERR_INVALID_ARG, "unknown norm type");
        const int tb = opts.batch_block_size ? opts.batch_block_size : 512;
        const BatchedFn fn = batched_fn(tb);
        if (!fn) return set_error(APCG_ERR_INVALID_ARG, "batch block size must be 256, 512 or 1024");
        if (!valid_batch_tail_rows(opts.batch_tail_tile_rows))
            return set_error(APCG_ERR_INVALID_ARG, "batch tail tile rows must be -1, 0 or a multiple of 256 in [256, 8192]");
        if (!valid_batch_tile_rows(opts.batch_tile_rows))
            return set_error(APCG_ERR_INVALID_ARG, "batch tile rows must be 0 or a multiple of 256 in [256, 8192]");
        const int dev = ctx->device;
        std::vector<BatchSys> hs(nsys);
        std::vector<double> cost(nsys);
        int64_t ws_total = 0;
        for (int32_t i = 0; i < nsys; ++i) {
            if (!A[i] || !b[i] || !x[i]) return set_error(APCG_ERR_INVALID_ARG, "NULL system handle");
            if (A[i]->device != dev || b[i]->device != dev || x[i]->device != dev || info->device != dev)
                return set_error(APCG_ERR_INVALID_ARG, "operands on different devices");
            if (b[i]->n != A[i]->n || x[i]->n != A[i]->n) return set_error(APCG_ERR_INVALID_ARG, "dimension mismatch");
            if (b[i] == x[i] || (b[i]->d == x[i]->d && A[i]->n > 0))
                return set_error(APCG_ERR_INVALID_ARG, "b and x must not alias");
            const int64_t n = A[i]->n;
            hs[i] = BatchSys{A[i]->rowptr, A[i]->col, A[i]->val, b[i]->d, x[i]->d, nullptr,
                             nullptr, nullptr, nullptr, (int32_t)n, 0};
            if (A[i]->cfg.schedule == APCG_SPMV_SDIA && A[i]->sdia_state == 1 && A[i]->sdia_mp == 8) {
                hs[i].soff = A[i]->sdia_off;
                hs[i].smask = A[i]->sdia_msk;
                hs[i].sval = A[i]->sdia_val;
                hs[i].U = A[i]->sdia_u;
            }
            hs[i].ws = reinterpret_cast<double *>(ws_total);  // offset for now
            ws_total += ((6 * n + 63) / 64) * 64;  // r, dinv, p0, p1, w, z (z: segmented schedule only)
            // CG iterations grow like sqrt(condition) ~ n^(1/2) in 2D (n^(1/3) in 3D):
            // estimated cost = nnz * sqrt(n)
            cost[i] = (double)(A[i]->nnz + n) * std::sqrt((double)std::max<int64_t>(n, 1));
        }
        if (apcg_status s = check_batch_ranges(nsys, b, x)) return s;
        std::vector<int32_t> order(nsys);
        std::iota(order.begin(), order.end(), 0);
        std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t c) { return cost[a] > cost[c]; });

        BatchCache *bc = batch_cache(ctx);
        // Ordering: x read-write, info written, A and b read
        std::vector<Acc> acc;
        acc.reserve(3 * nsys + 1);
        for (int32_t i = 0; i < nsys; ++i) {
            acc.push_back({&x[i]->rec, ACC_RW});
            acc.push_back({&A[i]->rec, ACC_R});
            acc.push_back({&b[i]->rec, ACC_R});
        }
        acc.push_back({&info->rec, ACC_W});
        apcg_status s;
        if ((s = op_begin(ctx, acc.data(), (int)acc.size()))) return s;
        hipStream_t st = ctx->stream;

        // (re)allocate device descriptors and workspace; the old buffers may
        // still be used by queued work, so their release is deferred
        if (bc->sys_cap < nsys || bc->ws_cap < ws_total) {
            EventRef ev = event_get(dev);
            if (!ev) return set_error(APCG_ERR_HIP, "event creation failed");
            APCG_HIP(hipEventRecord(ev->e, st));
            BatchCache old = *bc;
            defer_release({ev}, [old]() {
                hipSetDevice(old.device);
                if (old.exec) hipGraphExecDestroy(old.exec);
                if (old.graph) hipGraphDestroy(old.graph);
                hipFree(old.d_sys);
                hipFree(old.d_order);
                hipFree(old.d_queue);
                hipFree(old.d_ws);
            });
            bc->exec = nullptr;
            bc->graph = nullptr;
            bc->graph_hash = 0;
            bc->desc_hash = 0;
            const int64_t cap = std::max<int64_t>(nsys, bc->sys_cap);
            APCG_HIP(hipMalloc((void **)&bc->d_sys, sizeof(BatchSys) * cap));
            APCG_HIP(hipMalloc((void **)&bc->d_order, sizeof(int32_t) * cap));
            APCG_HIP(hipMalloc((void **)&bc->d_queue, 256));
            APCG_HIP(hipMalloc((void **)&bc->d_ws, sizeof(double) * std::max<int64_t>(ws_total, 64)));
            bc->sys_cap = cap;
            bc->ws_cap = std::max<int64_t>(ws_total, 64);
        }
        for (int32_t i = 0; i < nsys; ++i) hs[i].ws = bc->d_ws + reinterpret_cast<int64_t>(hs[i].ws);
        // refill the sliced-diagonal values of the systems that use them
        for (int32_t i = 0; i < nsys; ++i)
            if (hs[i].sval && (s = prepare_sdia(A[i], st))) return s;
        uint64_t h = fnv1a(hs.data(), sizeof(BatchSys) * nsys);
        h = fnv1a(order.data(), sizeof(int32_t) * nsys, h);
        if (h != bc->desc_hash) {
            g_counters.h2d_copies += 2;
            APCG_HIP(hipMemcpyAsync(bc->d_sys, hs.data(), sizeof(BatchSys) * nsys, hipMemcpyHostToDevice, st));
            APCG_HIP(hipMemcpyAsync(bc->d_order, order.data(), sizeof(int32_t) * nsys, hipMemcpyHostToDevice, st));
            // the host arrays are local: wait until the copies have consumed them
            g_counters.host_syncs++;
            APCG_HIP(hipStreamSynchronize(st));
            bc->desc_hash = h;
        }

        hipDeviceProp_t prop;
        APCG_HIP(hipGetDeviceProperties(&prop, dev));
        int sched = opts.batch_schedule;
        if (sched == APCG_BATCH_AUTO) {
            // one workgroup per system finishes no earlier than its costliest
            // system on one CU; the segmented schedule spreads every system
            // over the whole chip
            const double total = std::accumulate(cost.begin(), cost.end(), 0.0);
            const double worst = *std::max_element(cost.begin(), cost.end());
            sched = worst * prop.multiProcessorCount <= total ? APCG_BATCH_PERSISTENT : APCG_BATCH_SEGMENTED;
        }
        if (sched == APCG_BATCH_SEGMENTED) {
            if ((s = seg_solve(ctx, nsys, hs.data(), bc->d_sys, rtol, maxit, opts, info->d))) return s;
            return op_end(ctx, acc.data(), (int)acc.size());
        }
        if (sched != APCG_BATCH_PERSISTENT) return set_error(APCG_ERR_INVALID_ARG, "unknown batch schedule");
        int per_cu = 0;
        APCG_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void *>(fn), tb, 0));
        const int grid = std::max(1, std::min<int>(nsys, std::max(1, per_cu) * prop.multiProcessorCount));
        const int norm_pre = opts.norm_type == APCG_NORM_PRECONDITIONED;
        const int x0z = opts.x0_is_zero ? 1 : 0;

        uint64_t gh = fnv1a(&h, sizeof h);
        double params[2] = {rtol, (double)maxit};
        int iparams[6] = {grid, tb, x0z, opts.pc, norm_pre, nsys};
        gh = fnv1a(params, sizeof params, gh);
        gh = fnv1a(iparams, sizeof iparams, gh);
        const void *ip = info->d;
        gh = fnv1a(&ip, sizeof ip, gh);
        if (opts.mode == APCG_MODE_GRAPH) {
            if (!bc->exec || bc->graph_hash != gh) {
                if (bc->exec) {
                    EventRef ev = event_get(dev);
                    if (ev) hipEventRecord(ev->e, st);
                    hipGraphExec_t oe = bc->exec;
                    hipGraph_t og = bc->graph;
                    defer_release({ev}, [oe, og, dev]() {
                        hipSetDevice(dev);
                        hipGraphExecDestroy(oe);
                        hipGraphDestroy(og);
                    });
                    bc->exec = nullptr;
                    bc->graph = nullptr;
                }
                APCG_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeRelaxed));
                hipLaunchKernelGGL(k_queue_reset, dim3(1), dim3(64), 0, st, bc->d_queue);
                hipLaunchKernelGGL(fn, dim3(grid), dim3(tb), 0, st, (const BatchSys *)bc->d_sys,
                                   (const int32_t *)bc->d_order, nsys, bc->d_queue, rtol, maxit, x0z, opts.pc,
                                   norm_pre, info->d);
                hipGraph_t g = nullptr;
                hipError_t e = hipStreamEndCapture(st, &g);
                if (e != hipSuccess) return hip_error(e, "hipStreamEndCapture(batched)");
                e = hipGraphInstantiate(&bc->exec, g, nullptr, nullptr, 0);
                if (e != hipSuccess) {
                    hipGraphDestroy(g);
                    return hip_error(e, "hipGraphInstantiate(batched)");
                }
                bc->graph = g;
                bc->graph_hash = gh;
            }
            g_counters.graph_launches++;
            APCG_HIP(hipGraphLaunch(bc->exec, st));
        } else {
            hipLaunchKernelGGL(k_queue_reset, dim3(1), dim3(64), 0, st, bc->d_queue);
            APCG_CHECK_LAUNCH("k_queue_reset");
            hipLaunchKernelGGL(fn, dim3(grid), dim3(tb), 0, st, (const BatchSys *)bc->d_sys,
                               (const int32_t *)bc->d_order, nsys, bc->d_queue, rtol, maxit, x0z, opts.pc, norm_pre,
                               info->d);
            APCG_CHECK_LAUNCH("k_pcg_batched");
        }
        return op_end(ctx, acc.data(), (int)acc.size());
    } catch (const std::bad_alloc &) {
        return set_error(APCG_ERR_OUT_OF_MEMORY, "host allocation failed");
    }
}

// ===========================================================================
// Segmented schedule: the batch as one block-diagonal system.
//
// Rows of every system are cut into tiles of ST rows (a tile never crosses
// two systems).  Each iteration is four kernels, queued K iterations at a
// time in a captured graph:
//   seg_product (tiles):   p_new = D^-1 r + beta_s p_old, w = A p_new, and a
//                          partial of p.w per tile;
//   seg_alpha   (systems): one workgroup per system adds its tiles' partials
//                          in order, tests p.Ap, alpha_s = rho_s / delta_s;
//   seg_update  (tiles):   x += alpha_s p, r -= alpha_s w, partials of z.r
//                          and ||r||^2 per tile;
//   seg_beta    (systems): the tests of the iteration and beta_s.
// Every system keeps its own scalars and stop flag; tiles of stopped systems
// return at once, and a device count of running systems lets the host stop
// queueing graphs.  All CUs stream all systems' rows, so the batch runs at
// HBM speed instead of one CU per system.
// ===========================================================================

namespace apcg {

struct SegSys {  // per-system scalars, owned by the per-system kernels
    double rho, beta, alpha, delta;
    double res, ref;
    int32_t its, status, flag, zero_x;
};

// A tile is tile_rows rows of one system (a multiple of 256, starting at a
// multiple of tile_rows); its workgroup's four wavefronts take its 64-row
// slices in turn (wavefront j: slices j, j + 4, ...).  Partials are per
// slice: local slice l of system s is global slice sys_slice0[s] + l.  A
// wavefront adds its 64 rows and stores the slice's partial itself, so no
// tile kernel needs a workgroup barrier to reduce, and the per-system kernels
// add a system's slices in index order -- the same sums whatever the tile
// size.
struct SegPlan {
    const BatchSys *sys;   // [nsys]
    const int32_t *tile_sys, *tile_row0;  // [ntiles]
    const int32_t *sys_tile0;  // [nsys + 1]
    const int32_t *sys_slice0;  // [nsys + 1]
    SegSys *st;            // [nsys]
    double *part_res;      // [4][nslices]
    double *part_delta;    // [nslices]
    unsigned *running;     // [0]: systems still iterating; [2..3]: their rows (64-bit)
    int32_t nsys, ntiles, tiles_per_block;
    int32_t nslices;       // sys_slice0[nsys]
    int32_t tile_rows;
};

namespace {

// Rows of the systems still running, kept beside the count.
__device__ __forceinline__ unsigned long long *seg_running_rows(const SegPlan &P) {
    return reinterpret_cast<unsigned long long *>(P.running + 2);
}

constexpr int ST = 256;  // threads per tile workgroup (tiles are multiples of ST rows)
constexpr int SW = ST / 64;  // wavefronts per tile workgroup

// The local slices [sl0, sl1) of tile t (of a system of n rows).
__device__ __forceinline__ void tile_slices(const SegPlan &P, int t, int n, int *sl0, int *sl1) {
    const int r0 = P.tile_row0[t];
    *sl0 = r0 >> 6;
    *sl1 = min((n + 63) >> 6, (r0 + P.tile_rows) >> 6);
}

// Stores the calling wavefront's sums of v over its 64 rows as the partials
// of global slice g (partials[k * ns + g]); lane 0 stores.
template <int NV>
__device__ __forceinline__ void slice_store(double (&v)[NV], double *partials, int ns, int g) {
#pragma unroll
    for (int k = 0; k < NV; ++k) v[k] = dev::wave_sum(v[k]);
    if ((threadIdx.x & 63) == 0) {
#pragma unroll
        for (int k = 0; k < NV; ++k) partials[(int64_t)k * ns + g] = v[k];
    }
}

// Runs body(t) for every tile t of this workgroup whose system passes
// keep(state).  Workgroup lb (its XCD-aware index) owns tiles lb, lb + G,
// lb + 2G, ...: a system's consecutive tiles go to different workgroups, so
// when only a few systems are still running their tiles are worked on side
// by side rather than one after another by a few workgroups, and each round
// of G tiles is split into eight contiguous runs, one per XCD.  Tiles are
// screened ST at a time (one per thread) and the survivors compacted in
// LDS, so the tiles of stopped systems cost one round of loads per ST tiles.
// Each tile writes only its own outputs.
template <typename Keep, typename Body>
__device__ __forceinline__ void for_active_tiles(const SegPlan &P, Keep keep, Body body) {
    const int lb = dev::xcd_block(blockIdx.x, gridDim.x), G = gridDim.x;
    __shared__ int list[ST];
    __shared__ int cnt;
    for (int base = 0; lb + base * G < P.ntiles; base += ST) {
        if (threadIdx.x == 0) cnt = 0;
        __syncthreads();
        const int t = lb + (base + (int)threadIdx.x) * G;
        if (t < P.ntiles && keep(P.st[P.tile_sys[t]])) list[atomicAdd(&cnt, 1)] = t;
        __syncthreads();
        const int m = cnt;
        for (int k = 0; k < m; ++k) body(__builtin_amdgcn_readfirstlane(list[k]));
        __syncthreads();  // the list is reused by the next round
    }
}

__global__ __launch_bounds__(ST) void k_seg_init(SegPlan P, int x0_zero, int pc, int norm_pre) {
    const int tb0 = dev::xcd_block(blockIdx.x, gridDim.x), tstep = gridDim.x;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    for (int t = tb0; t < P.ntiles; t += tstep) {
      const int sys = P.tile_sys[t];
      const BatchSys S = P.sys[sys];
      int sl0, sl1;
      tile_slices(P, t, S.n, &sl0, &sl1);
      for (int sl = sl0 + wave; sl < sl1; sl += SW) {
        const int i = sl * 64 + lane;
        double v[4] = {0.0, 0.0, 0.0, 0.0};
        if (i < S.n) {
            const int s = S.rowptr[i], e = S.rowptr[i + 1];
            double diag = 0.0, ax = 0.0;
            bool found = false;
            for (int k = s; k < e; ++k) {
                const int j = S.col[k];
                const double a = S.val[k];
                if (j == i) {
                    diag = a;
                    found = true;
                }
                if (!x0_zero) ax = fma(a, S.x[j], ax);
            }
            double di = 1.0;
            if (pc == APCG_PC_JACOBI) {
                const bool ok = found && diag > 0.0;
                v[3] = ok ? 0.0 : 1.0;
                di = ok ? 1.0 / diag : 0.0;
            }
            const double bi = S.b[i];
            const double ri = x0_zero ? bi : bi - ax;
            const int64_t n = S.n;
            S.ws[i] = ri;             // r
            S.ws[n + i] = di;         // dinv
            S.ws[2 * n + i] = 0.0;    // p[0]
            if (x0_zero) S.x[i] = 0.0;
            const double zi = di * ri;
            S.ws[5 * n + i] = zi;     // z
            v[0] = zi * ri;
            if (norm_pre) {
                const double zb = di * bi;
                v[1] = zi * zi;
                v[2] = zb * zb;
            } else {
                v[1] = ri * ri;
                v[2] = bi * bi;
            }
        }
        slice_store<4>(v, P.part_res, P.nslices, P.sys_slice0[sys] + sl);
      }
    }
}

// Threads of the per-system kernels (one workgroup per system).
constexpr int SB = 256;

// Adds the slice partials part[k*ns + g] of a system (its slices ga..gb)
// in a fixed order: thread l takes g = ga + l, ga + l + SB, ..., then the
// workgroup tree.  Result in thread 0.
template <int NV>
__device__ __forceinline__ void sys_sum(const double *part, int ns, int ga, int gb, double (&v)[NV], double *lds) {
#pragma unroll
    for (int k = 0; k < NV; ++k) v[k] = 0.0;
    int g = ga + (int)threadIdx.x;
    // eight of a thread's partials loaded before they are added (a large
    // system has thousands of slices); the same order of addition
    constexpr int UA = 8;
    for (; g + (UA - 1) * SB < gb; g += UA * SB) {
        double t[UA][NV];
#pragma unroll
        for (int u = 0; u < UA; ++u)
#pragma unroll
            for (int k = 0; k < NV; ++k) t[u][k] = part[(int64_t)k * ns + g + u * SB];
#pragma unroll
        for (int u = 0; u < UA; ++u)
#pragma unroll
            for (int k = 0; k < NV; ++k) v[k] += t[u][k];
    }
    for (; g < gb; g += SB) {
#pragma unroll
        for (int k = 0; k < NV; ++k) v[k] += part[(int64_t)k * ns + g];
    }
    dev::block_sum<SB, NV>(v, lds);
}

__global__ __launch_bounds__(SB) void k_seg_init_final(SegPlan P, double rtol, int32_t maxit) {
    const int s = blockIdx.x;
    __shared__ double lds[4 * (SB / 64)];
    double v[4];
    sys_sum<4>(P.part_res, P.nslices, P.sys_slice0[s], P.sys_slice0[s + 1], v, lds);
    if (threadIdx.x != 0) return;
    SegSys q;
    q.rho = v[0];
    q.res = sqrt(v[1]);
    q.ref = sqrt(v[2]);
    q.beta = 0.0;
    q.alpha = 0.0;
    q.delta = 0.0;
    q.its = 0;
    q.zero_x = 0;
    int status = 0;
    if (v[3] > 0.0) status = APCG_SOLVE_SETUP_ERROR;
    else if (q.ref == 0.0) {
        status = APCG_SOLVE_CONVERGED;
        q.zero_x = 1;
        q.res = 0.0;
    } else if (!isfinite(q.res) || !isfinite(q.ref)) status = APCG_SOLVE_NAN;
    else if (q.res <= rtol * q.ref) status = APCG_SOLVE_CONVERGED;
    else if (!(q.rho > 0.0)) status = isfinite(q.rho) ? APCG_SOLVE_BREAKDOWN_RZ : APCG_SOLVE_NAN;
    else if (maxit <= 0) status = APCG_SOLVE_MAXIT;
    q.status = status;
    q.flag = status != 0;
    P.st[s] = q;
    if (!q.flag) {
        atomicAdd(P.running, 1u);
        atomicAdd(seg_running_rows(P), (unsigned long long)P.sys[s].n);
    }
}

__global__ __launch_bounds__(ST) void k_seg_zero_x(SegPlan P) {
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    for_active_tiles(P, [](const SegSys &q) { return q.zero_x != 0; }, [&](int t) {
        const BatchSys S = P.sys[P.tile_sys[t]];
        int sl0, sl1;
        tile_slices(P, t, S.n, &sl0, &sl1);
        for (int sl = sl0 + wave; sl < sl1; sl += SW) {
            const int i = sl * 64 + lane;
            if (i < S.n) S.x[i] = 0.0;
        }
    });
}

// UC: sliced-diagonal slots walked per row (>= every such system's U).
template <int UC>
__global__ __launch_bounds__(ST) void k_seg_product(SegPlan P, int parity) {
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    for_active_tiles(P, [](const SegSys &q) { return !q.flag; }, [&](int t) {
        const int s = P.tile_sys[t];
        const double beta = P.st[s].beta;
        const BatchSys S = P.sys[s];
        const int64_t n = S.n;
        const auto *z = dev::glb(S.ws + 5 * n);
        const auto *pold = dev::glb(S.ws + (2 + ((parity + 1) & 1)) * n);
        auto *pnew = dev::glb(S.ws + (2 + (parity & 1)) * n);
        auto *w = dev::glb(S.ws + 4 * n);
        const int g0 = P.sys_slice0[s];
        int sl0, sl1;
        tile_slices(P, t, S.n, &sl0, &sl1);
        if (S.sval) {  // the next slice's offsets and values loaded during the current gathers
            auto u = [&](int q) { return fma(beta, pold[q], z[q]); };
            auto f = [&](int sl, int row, int rc, double sum) {
                const double pi = fma(beta, pold[rc], z[rc]);
                double v[1] = {0.0};
                if (row < n) {
                    pnew[row] = pi;
                    w[row] = sum;
                    v[0] = pi * sum;
                }
                slice_store<1>(v, P.part_delta, P.nslices, g0 + sl);
            };
            dev::sdia_slices<UC>(S.soff, S.smask, S.sval, S.U, n, sl0 + wave, sl1, SW, u, f);
            return;
        }
        for (int sl = sl0 + wave; sl < sl1; sl += SW) {
            const int i = sl * 64 + lane;
            double v[1] = {0.0};
            if (i < S.n) {
                const auto *rp = dev::glb(S.rowptr);
                const double sum = row_product_z(dev::glb(S.col), dev::glb(S.val), rp[i], rp[i + 1], i, z, pold, beta);
                const double pi = fma(beta, pold[i], z[i]);
                pnew[i] = pi;
                w[i] = sum;
                v[0] = pi * sum;
            }
            slice_store<1>(v, P.part_delta, P.nslices, g0 + sl);
        }
    });
}

__global__ __launch_bounds__(SB) void k_seg_alpha(SegPlan P) {
    const int s = blockIdx.x;
    if (P.st[s].flag) return;
    __shared__ double lds[1 * (SB / 64)];
    double v[1];
    sys_sum<1>(P.part_delta, P.nslices, P.sys_slice0[s], P.sys_slice0[s + 1], v, lds);
    if (threadIdx.x != 0) return;
    SegSys *q = P.st + s;
    const double delta = v[0];
    q->delta = delta;
    if (!(delta > 0.0)) {
        q->status = isfinite(delta) ? APCG_SOLVE_BREAKDOWN_PAP : APCG_SOLVE_NAN;
        q->flag = 1;
        atomicSub(P.running, 1u);
        atomicAdd(seg_running_rows(P), 0ull - (unsigned long long)P.sys[s].n);
    } else {
        q->alpha = q->rho / delta;
    }
}

__global__ __launch_bounds__(ST) void k_seg_update(SegPlan P, int parity, int norm_pre) {
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    for_active_tiles(P, [](const SegSys &q) { return !q.flag; }, [&](int t) {
      const int s = P.tile_sys[t];
      const double alpha = P.st[s].alpha;
      const BatchSys S = P.sys[s];
      const int64_t n = S.n;
      auto *r = dev::glb(S.ws);
      const auto *dinv = dev::glb(S.ws + n);
      const auto *p = dev::glb(S.ws + (2 + (parity & 1)) * n);
      const auto *w = dev::glb(S.ws + 4 * n);
      auto *x = dev::glb(S.x);
      auto *z = dev::glb(S.ws + 5 * n);
      const int g0 = P.sys_slice0[s];
      int sl0, sl1;
      tile_slices(P, t, S.n, &sl0, &sl1);
      // the wavefront's slices in groups of UN whose loads are all issued
      // before the group's arithmetic and stores (each slice's partials are
      // its own 64 rows' sums, as one slice at a time)
      constexpr int UN = 4;
      for (int sb = sl0 + wave; sb < sl1; sb += UN * SW) {
        double xs[UN], rs[UN], ps[UN], ws[UN], ds[UN];
#pragma unroll
        for (int u = 0; u < UN; ++u) {
          const int i = (sb + u * SW) * 64 + lane;
          const bool ok = sb + u * SW < sl1 && i < S.n;
          const int ic = ok ? i : 0;
          xs[u] = x[ic];
          rs[u] = r[ic];
          ps[u] = p[ic];
          ws[u] = w[ic];
          ds[u] = dinv[ic];
        }
#pragma unroll
        for (int u = 0; u < UN; ++u) {
          const int sl = sb + u * SW;
          if (sl >= sl1) break;
          const int i = sl * 64 + lane;
          double v[2] = {0.0, 0.0};
          if (i < S.n) {
            const double xi = fma(alpha, ps[u], xs[u]);
            const double ri = fma(-alpha, ws[u], rs[u]);
            x[i] = xi;
            r[i] = ri;
            const double zi = ds[u] * ri;
            z[i] = zi;  // gathered by the next product
            v[0] = zi * ri;
            v[1] = norm_pre ? zi * zi : ri * ri;
          }
          slice_store<2>(v, P.part_res, P.nslices, g0 + sl);
        }
      }
    });
}

__global__ __launch_bounds__(SB) void k_seg_beta(SegPlan P, double rtol, int32_t maxit) {
    const int s = blockIdx.x;
    if (P.st[s].flag) return;
    __shared__ double lds[2 * (SB / 64)];
    double v[2];
    sys_sum<2>(P.part_res, P.nslices, P.sys_slice0[s], P.sys_slice0[s + 1], v, lds);
    if (threadIdx.x != 0) return;
    SegSys *q = P.st + s;
    const double rho_new = v[0], res = sqrt(v[1]);
    const int its = q->its + 1;
    q->its = its;
    q->res = res;
    int status = 0;
    if (!isfinite(res) || !isfinite(rho_new)) status = APCG_SOLVE_NAN;
    else if (res <= rtol * q->ref) status = APCG_SOLVE_CONVERGED;
    else if (!(rho_new > 0.0)) status = APCG_SOLVE_BREAKDOWN_RZ;
    else if (its >= maxit) status = APCG_SOLVE_MAXIT;
    if (status) {
        q->status = status;
        q->flag = 1;
        atomicSub(P.running, 1u);
        atomicAdd(seg_running_rows(P), 0ull - (unsigned long long)P.sys[s].n);
    } else {
        q->beta = rho_new / q->rho;
        q->rho = rho_new;
    }
}

__global__ void k_seg_finish(SegPlan P, apcg_solve_info *info) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= P.nsys) return;
    const SegSys q = P.st[s];
    info[s].iterations = q.its;
    info[s].status = q.status ? q.status : APCG_SOLVE_MAXIT;
    info[s].fcg_iterations = 0;
    info[s].half_steps = 0;
    info[s].res_norm = q.res;
    info[s].ref_norm = q.ref;
}

__global__ void k_seg_reset(unsigned *running) {
    if (threadIdx.x < 4) running[threadIdx.x] = 0u;  // the count and the 64-bit row total
}

}  // namespace

// The tail plan of the segmented PCG takes over once the rows still running
// fill fewer than this many of the large tiles per compute unit.  Unlike the
// flexible iteration's (32), it stays low: the 2D batch (1024-row tiles, a
// 256-row tail) took 159.8 ms at 2 or without the switch, 160.1 at 8 and
// 216.4 at 32, where most of the solve runs on the small tiles.
constexpr uint64_t kSegTailTilesPerCu = 2;

// Segment resources of one context (tile tables, per-system scalars, graph).
struct SegCache {
    int device = 0;
    int32_t *d_tile_sys = nullptr, *d_tile_row0 = nullptr, *d_sys_tile0 = nullptr, *d_sys_slice0 = nullptr;
    SegSys *d_st = nullptr;
    double *d_part = nullptr;  // 5 * slices_cap (slice partials)
    unsigned *d_running = nullptr;
    int64_t tiles_cap = 0, sys_cap = 0, slices_cap = 0;
    uint64_t hash = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    uint64_t graph_hash = 0;
    // the tail plan: smaller tiles once few rows still run
    int32_t *d_tile_sys_t = nullptr, *d_tile_row0_t = nullptr;
    int64_t tiles_t_cap = 0;
    uint64_t hash_t = 0;
    hipGraph_t graph_t = nullptr;
    hipGraphExec_t exec_t = nullptr;
    uint64_t graph_hash_t = 0;
    int32_t cus = 0;            // compute units of the device
    int32_t *pinned = nullptr;  // [kMaxLookahead][4]: running count, pad, running rows (64-bit)
    EventRef poll_ev[kMaxLookahead];
};

static std::mutex g_seg_mu;
static std::vector<std::pair<uint64_t, SegCache *>> g_seg;

static SegCache *seg_cache(apcg_ctx c) {
    std::lock_guard<std::mutex> lk(g_seg_mu);
    for (auto &p : g_seg)
        if (p.first == c->id) return p.second;
    SegCache *sc = new SegCache();
    sc->device = c->device;
    g_seg.emplace_back(c->id, sc);
    return sc;
}

static void seg_free_tail(SegCache &s) {
    if (s.exec_t) hipGraphExecDestroy(s.exec_t);
    if (s.graph_t) hipGraphDestroy(s.graph_t);
    hipFree(s.d_tile_sys_t);
    hipFree(s.d_tile_row0_t);
}

static void seg_free_buffers(SegCache &s) {
    if (s.exec) hipGraphExecDestroy(s.exec);
    if (s.graph) hipGraphDestroy(s.graph);
    hipFree(s.d_tile_sys);
    hipFree(s.d_tile_row0);
    hipFree(s.d_sys_tile0);
    hipFree(s.d_sys_slice0);
    hipFree(s.d_st);
    hipFree(s.d_part);
    hipFree(s.d_running);
}

void seg_cache_release(uint64_t ctx_id, int device) {
    SegCache *sc = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_seg_mu);
        for (auto it = g_seg.begin(); it != g_seg.end(); ++it)
            if (it->first == ctx_id) {
                sc = it->second;
                g_seg.erase(it);
                break;
            }
    }
    if (!sc) return;
    hipSetDevice(device);
    seg_free_buffers(*sc);
    seg_free_tail(*sc);
    if (sc->pinned) hipHostFree(sc->pinned);
    delete sc;
}

// Enqueues the segmented solve of the batch whose descriptors are already on
// the device (d_sys).  Called from apcg_ksp_solve_batched.
apcg_status seg_solve(apcg_ctx ctx, int32_t nsys, const BatchSys *hsys, const BatchSys *d_sys, double rtol,
                      int32_t maxit, const apcg_solve_opts &opts, apcg_solve_info *d_info) {
    SegCache *sc = seg_cache(ctx);
    const int dev = ctx->device;
    hipStream_t st = ctx->stream;
    const int32_t TR = batch_tile_rows(opts);
    std::vector<int32_t> tile_sys, tile_row0, sys_tile0(nsys + 1), sys_slice0(nsys + 1);
    int64_t nslices = 0;
    for (int32_t s = 0; s < nsys; ++s) {
        sys_tile0[s] = (int32_t)tile_sys.size();
        sys_slice0[s] = (int32_t)nslices;
        const int32_t n = hsys[s].n;
        nslices += ((int64_t)n + 63) / 64;
        for (int32_t r0 = 0; r0 < n; r0 += TR) {
            tile_sys.push_back(s);
            tile_row0.push_back(r0);
        }
    }
    sys_tile0[nsys] = (int32_t)tile_sys.size();
    sys_slice0[nsys] = (int32_t)nslices;
    if (nslices > INT32_MAX / 8) return set_error(APCG_ERR_INVALID_ARG, "batch too large for the segmented schedule");
    // the tail plan: the same systems in smaller tiles, switched to once the
    // rows still running fill fewer than two of the large tiles per compute
    // unit (the tiles only group slices, so the sums are those of the
    // large tiles)
    const int32_t TRt = batch_tail_rows(opts);
    std::vector<int32_t> tile_sys_t, tile_row0_t;
    if (TRt > 0)
        for (int32_t s = 0; s < nsys; ++s)
            for (int32_t r0 = 0; r0 < hsys[s].n; r0 += TRt) {
                tile_sys_t.push_back(s);
                tile_row0_t.push_back(r0);
            }
    const int32_t ntiles_t = (int32_t)tile_sys_t.size();
    const bool tail_plan = ntiles_t > 0;
    const int64_t ns_alloc = std::max<int64_t>(nslices, 1);
    const int32_t ntiles = (int32_t)tile_sys.size();
    if (ntiles == 0) {  // every system is empty: one dummy tile keeps the kernels well-formed
        tile_sys.push_back(0);
        tile_row0.push_back(0);
    }
    const int32_t nt_alloc = std::max<int32_t>(ntiles, 1);
    if (sc->tiles_cap < nt_alloc || sc->sys_cap < nsys || sc->slices_cap < ns_alloc) {
        EventRef ev = event_get(dev);
        if (!ev) return set_error(APCG_ERR_HIP, "event creation failed");
        APCG_HIP(hipEventRecord(ev->e, st));
        SegCache old = *sc;
        defer_release({ev}, [old, dev]() mutable {
            hipSetDevice(dev);
            seg_free_buffers(old);
        });
        sc->exec = nullptr;
        sc->graph = nullptr;
        sc->graph_hash = 0;
        sc->hash = 0;
        sc->tiles_cap = std::max<int64_t>(nt_alloc, sc->tiles_cap);
        sc->slices_cap = std::max<int64_t>(ns_alloc, sc->slices_cap);
        sc->sys_cap = std::max<int64_t>(nsys, sc->sys_cap);
        APCG_HIP(hipMalloc((void **)&sc->d_tile_sys, sizeof(int32_t) * sc->tiles_cap));
        APCG_HIP(hipMalloc((void **)&sc->d_tile_row0, sizeof(int32_t) * sc->tiles_cap));
        APCG_HIP(hipMalloc((void **)&sc->d_sys_tile0, sizeof(int32_t) * (sc->sys_cap + 1)));
        APCG_HIP(hipMalloc((void **)&sc->d_sys_slice0, sizeof(int32_t) * (sc->sys_cap + 1)));
        APCG_HIP(hipMalloc((void **)&sc->d_st, sizeof(SegSys) * sc->sys_cap));
        APCG_HIP(hipMalloc((void **)&sc->d_part, sizeof(double) * 5 * sc->slices_cap));
        APCG_HIP(hipMalloc((void **)&sc->d_running, 256));
    }
    if (!sc->pinned)
        APCG_HIP(hipHostMalloc((void **)&sc->pinned, sizeof(int32_t) * 4 * kMaxLookahead, hipHostMallocDefault));
    uint64_t h = fnv1a(tile_sys.data(), sizeof(int32_t) * tile_sys.size());
    h = fnv1a(tile_row0.data(), sizeof(int32_t) * tile_row0.size(), h);
    h = fnv1a(sys_tile0.data(), sizeof(int32_t) * sys_tile0.size(), h);
    h = fnv1a(sys_slice0.data(), sizeof(int32_t) * sys_slice0.size(), h);
    if (h != sc->hash) {
        g_counters.h2d_copies += 4;
        APCG_HIP(hipMemcpyAsync(sc->d_tile_sys, tile_sys.data(), sizeof(int32_t) * tile_sys.size(),
                                hipMemcpyHostToDevice, st));
        APCG_HIP(hipMemcpyAsync(sc->d_tile_row0, tile_row0.data(), sizeof(int32_t) * tile_row0.size(),
                                hipMemcpyHostToDevice, st));
        APCG_HIP(hipMemcpyAsync(sc->d_sys_tile0, sys_tile0.data(), sizeof(int32_t) * sys_tile0.size(),
                                hipMemcpyHostToDevice, st));
        APCG_HIP(hipMemcpyAsync(sc->d_sys_slice0, sys_slice0.data(), sizeof(int32_t) * sys_slice0.size(),
                                hipMemcpyHostToDevice, st));
        g_counters.host_syncs++;
        APCG_HIP(hipStreamSynchronize(st));  // host tables are local
        sc->hash = h;
    }
    if (tail_plan) {
        if (sc->tiles_t_cap < ntiles_t) {
            EventRef ev = event_get(dev);
            if (!ev) return set_error(APCG_ERR_HIP, "event creation failed");
            APCG_HIP(hipEventRecord(ev->e, st));
            SegCache old = *sc;
            defer_release({ev}, [old, dev]() mutable {
                hipSetDevice(dev);
                seg_free_tail(old);
            });
            sc->exec_t = nullptr;
            sc->graph_t = nullptr;
            sc->graph_hash_t = 0;
            sc->hash_t = 0;
            sc->tiles_t_cap = ntiles_t;
            APCG_HIP(hipMalloc((void **)&sc->d_tile_sys_t, sizeof(int32_t) * sc->tiles_t_cap));
            APCG_HIP(hipMalloc((void **)&sc->d_tile_row0_t, sizeof(int32_t) * sc->tiles_t_cap));
        }
        uint64_t ht = fnv1a(tile_sys_t.data(), sizeof(int32_t) * tile_sys_t.size());
        ht = fnv1a(tile_row0_t.data(), sizeof(int32_t) * tile_row0_t.size(), ht);
        if (ht != sc->hash_t) {
            g_counters.h2d_copies += 2;
            APCG_HIP(hipMemcpyAsync(sc->d_tile_sys_t, tile_sys_t.data(), sizeof(int32_t) * tile_sys_t.size(),
                                    hipMemcpyHostToDevice, st));
            APCG_HIP(hipMemcpyAsync(sc->d_tile_row0_t, tile_row0_t.data(), sizeof(int32_t) * tile_row0_t.size(),
                                    hipMemcpyHostToDevice, st));
            g_counters.host_syncs++;
            APCG_HIP(hipStreamSynchronize(st));  // host tables are local
            sc->hash_t = ht;
        }
        if (!sc->cus) APCG_HIP(hipDeviceGetAttribute(&sc->cus, hipDeviceAttributeMultiprocessorCount, dev));
    }
    SegPlan P;
    P.sys = d_sys;
    P.tile_sys = sc->d_tile_sys;
    P.tile_row0 = sc->d_tile_row0;
    P.sys_tile0 = sc->d_sys_tile0;
    P.sys_slice0 = sc->d_sys_slice0;
    P.st = sc->d_st;
    P.part_res = sc->d_part;
    P.part_delta = sc->d_part + 4 * sc->slices_cap;
    P.running = sc->d_running;
    P.nsys = nsys;
    P.ntiles = ntiles;
    P.nslices = (int32_t)ns_alloc;
    P.tile_rows = TR;
    const int G = normalise_blocks(kMaxBlocks, std::max<int32_t>(ntiles, 1));  // few tiles per workgroup: more in flight
    P.tiles_per_block = std::max<int32_t>(1, (ntiles + G - 1) / G);
    SegPlan Pt = P;
    int Gt = G;
    if (tail_plan) {
        Pt.tile_sys = sc->d_tile_sys_t;
        Pt.tile_row0 = sc->d_tile_row0_t;
        Pt.ntiles = ntiles_t;
        Pt.tile_rows = TRt;
        Gt = normalise_blocks(kMaxBlocks, ntiles_t);
        Pt.tiles_per_block = std::max<int32_t>(1, (ntiles_t + Gt - 1) / Gt);
    }
    // switch when the running rows fill fewer than kSegTailTilesPerCu large tiles per CU
    const uint64_t tail_rows = tail_plan ? kSegTailTilesPerCu * (uint64_t)sc->cus * (uint64_t)TR : 0;
    const int norm_pre = opts.norm_type == APCG_NORM_PRECONDITIONED;
    const int x0z = opts.x0_is_zero ? 1 : 0;

    hipLaunchKernelGGL(k_seg_reset, dim3(1), dim3(64), 0, st, sc->d_running);
    APCG_CHECK_LAUNCH("k_seg_reset");
    hipLaunchKernelGGL(k_seg_init, dim3(G), dim3(ST), 0, st, P, x0z, opts.pc, norm_pre);
    APCG_CHECK_LAUNCH("k_seg_init");
    hipLaunchKernelGGL(k_seg_init_final, dim3(nsys), dim3(SB), 0, st, P, rtol, maxit);
    APCG_CHECK_LAUNCH("k_seg_init_final");
    hipLaunchKernelGGL(k_seg_zero_x, dim3(G), dim3(ST), 0, st, P);
    APCG_CHECK_LAUNCH("k_seg_zero_x");

    int K = std::max(2, opts.iters_per_graph);
    if (K & 1) ++K;
    const int L = std::max(1, std::min(kMaxLookahead, opts.lookahead));
    int umax = 0;  // most sliced-diagonal slots of any system that reads them
    for (int32_t i = 0; i < nsys; ++i)
        if (hsys[i].sval) umax = std::max<int>(umax, hsys[i].U);
    void (*seg_product)(SegPlan, int) = umax <= 5   ? k_seg_product<5>
                                        : umax <= 7 ? k_seg_product<7>
                                                    : k_seg_product<8>;
    auto launch_iter = [&](int j, const SegPlan &P, int G) -> apcg_status {
        hipLaunchKernelGGL(seg_product, dim3(G), dim3(ST), 0, st, P, j & 1);
        APCG_CHECK_LAUNCH("k_seg_product");
        hipLaunchKernelGGL(k_seg_alpha, dim3(nsys), dim3(SB), 0, st, P);
        APCG_CHECK_LAUNCH("k_seg_alpha");
        hipLaunchKernelGGL(k_seg_update, dim3(G), dim3(ST), 0, st, P, j & 1, norm_pre);
        APCG_CHECK_LAUNCH("k_seg_update");
        hipLaunchKernelGGL(k_seg_beta, dim3(nsys), dim3(SB), 0, st, P, rtol, maxit);
        APCG_CHECK_LAUNCH("k_seg_beta");
        return APCG_SUCCESS;
    };
    // K iterations of plan Pc on grid Gc captured into one executable graph
    auto capture = [&](const SegPlan &Pc, int Gc, hipGraph_t *gout, hipGraphExec_t *xout) -> apcg_status {
        APCG_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeRelaxed));
        apcg_status cs = APCG_SUCCESS;
        for (int j = 1; j <= K && cs == APCG_SUCCESS; ++j) cs = launch_iter(j, Pc, Gc);
        hipGraph_t g = nullptr;
        hipError_t e = hipStreamEndCapture(st, &g);
        if (cs) {
            if (g) hipGraphDestroy(g);
            return cs;
        }
        if (e != hipSuccess) return hip_error(e, "hipStreamEndCapture(segmented)");
        g_counters.kernel_launches -= 4 * K;
        e = hipGraphInstantiate(xout, g, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            hipGraphDestroy(g);
            return hip_error(e, "hipGraphInstantiate(segmented)");
        }
        *gout = g;
        return APCG_SUCCESS;
    };
    uint64_t gh = fnv1a(&h, sizeof h);
    const void *dsp = d_sys;
    gh = fnv1a(&dsp, sizeof dsp, gh);
    double prm[1] = {rtol};
    const int uc = umax <= 5 ? 5 : umax <= 7 ? 7 : 8;  // which tile product the graph holds
    int iprm[6] = {K, maxit, norm_pre, G, nsys, uc};
    gh = fnv1a(prm, sizeof prm, gh);
    gh = fnv1a(iprm, sizeof iprm, gh);
    apcg_status s;
    if (maxit > 0) {
        if (opts.mode == APCG_MODE_GRAPH) {
            if (!sc->exec || sc->graph_hash != gh) {
                if (sc->exec) {
                    EventRef ev = event_get(dev);
                    if (ev) hipEventRecord(ev->e, st);
                    hipGraphExec_t oe = sc->exec;
                    hipGraph_t og = sc->graph;
                    defer_release({ev}, [oe, og, dev]() {
                        hipSetDevice(dev);
                        hipGraphExecDestroy(oe);
                        hipGraphDestroy(og);
                    });
                    sc->exec = nullptr;
                    sc->graph = nullptr;
                }
                if ((s = capture(P, G, &sc->graph, &sc->exec))) return s;
                sc->graph_hash = gh;
            }
            // the tail plan's period, captured alike
            uint64_t ght = fnv1a(&sc->hash_t, sizeof sc->hash_t, gh);
            const int tprm[3] = {Gt, TRt, Pt.tiles_per_block};
            ght = fnv1a(tprm, sizeof tprm, ght);
            const void *tptrs[2] = {sc->d_tile_sys_t, sc->d_tile_row0_t};
            ght = fnv1a(tptrs, sizeof tptrs, ght);
            if (tail_plan && (!sc->exec_t || sc->graph_hash_t != ght)) {
                if (sc->exec_t) {
                    EventRef ev = event_get(dev);
                    if (ev) hipEventRecord(ev->e, st);
                    hipGraphExec_t oe = sc->exec_t;
                    hipGraph_t og = sc->graph_t;
                    defer_release({ev}, [oe, og, dev]() {
                        hipSetDevice(dev);
                        hipGraphExecDestroy(oe);
                        hipGraphDestroy(og);
                    });
                    sc->exec_t = nullptr;
                    sc->graph_t = nullptr;
                }
                if ((s = capture(Pt, Gt, &sc->graph_t, &sc->exec_t))) return s;
                sc->graph_hash_t = ght;
            }
        }
        const int64_t periods = ((int64_t)maxit + K - 1) / K;
        bool tail = false;  // periods on the tail plan from here on
        for (int64_t g = 0; g < periods; ++g) {
            if (opts.mode == APCG_MODE_GRAPH) {
                g_counters.graph_launches++;
                APCG_HIP(hipGraphLaunch(tail ? sc->exec_t : sc->exec, st));
            } else {
                for (int j = 1; j <= K; ++j)
                    if ((s = launch_iter(j, tail ? Pt : P, tail ? Gt : G))) return s;
            }
            const int slot = (int)(g % L);
            if (!sc->poll_ev[slot]) {
                sc->poll_ev[slot] = event_get(dev);
                if (!sc->poll_ev[slot]) return set_error(APCG_ERR_HIP, "event creation failed");
            }
            g_counters.d2h_copies++;
            APCG_HIP(hipMemcpyAsync(&sc->pinned[4 * slot], sc->d_running, 4 * sizeof(int32_t), hipMemcpyDeviceToHost,
                                    st));
            APCG_HIP(hipEventRecord(sc->poll_ev[slot]->e, st));
            if (g >= L - 1) {
                const int ps = (int)((g - (L - 1)) % L);
                g_counters.host_polls++;
                APCG_HIP(hipEventSynchronize(sc->poll_ev[ps]->e));
                if (sc->pinned[4 * ps] == 0) break;  // every system has stopped
                uint64_t rows;
                memcpy(&rows, &sc->pinned[4 * ps + 2], sizeof rows);
                if (tail_plan && !tail && rows < tail_rows) tail = true;
            }
        }
    }
    hipLaunchKernelGGL(k_seg_finish, dim3((nsys + 63) / 64), dim3(64), 0, st, P, d_info);
    APCG_CHECK_LAUNCH("k_seg_finish");
    return APCG_SUCCESS;
}

}  // namespace apcg
