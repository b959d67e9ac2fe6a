// batched_fcg.hip -- many FCG(1) solves, each with its own Chebyshev-basis
// polynomial preconditioner and its own fallback to Jacobi-PCG, run as one
// segmented (block-diagonal) iteration.
//
// Rows of every system are cut into tiles of FT rows (a tile never crosses
// two systems).  One iteration is thirteen kernels, K iterations per
// captured graph:
//   product (tiles)   p = z + beta_s p_old, w = A p, a partial of p.w per tile
//   alpha   (systems) delta_s from the tiles in order; p.w <= 0 is a breakdown
//   update  (tiles)   x += alpha_s p, r -= alpha_s w, a partial of ||r||^2
//   check   (systems) convergence, stall window and iteration cap
//   cheb x8 (tiles)   Clenshaw steps of z = p_s(D^-1 A) D^-1 r (a system in
//                     Jacobi mode only forms z = D^-1 r in the last step);
//                     the last writes partials of r.z and z.w
//   beta    (systems) FCG(1): beta = -(z.w) / delta; Jacobi mode: the PCG
//                     beta = (r.z)_new / (r.z)_old; r.z <= 0 is a breakdown
// A system switches to Jacobi mode -- continuing from its current x with a
// fresh direction -- when its polynomial is not positive on [0, lmax]
// (checked first, on 1024 points), on a breakdown, or on a stall, if the
// fallback is enabled.  A switch, and the first application of the
// preconditioner, take one "restart" slot: the product, alpha, update and
// check skip the system, the Clenshaw kernels form its z and the beta kernel
// starts its recurrence (beta = 0).  Per-system kernels own the per-system
// state; tile kernels only read it.  A device count of running systems lets
// the host stop queueing graphs.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "internal.h"

namespace apcg {
namespace {

constexpr int FT = 256;  // threads per tile workgroup (tiles are multiples of FT rows)
constexpr int FSW = FT / 64;  // its wavefronts: wavefront j takes slices j, j + 4, ... of a tile

constexpr int FDEG = 8;
constexpr int MODE_FLEX = 0, MODE_JACOBI = 1;

struct FSys {
    const int32_t *rowptr;
    const int32_t *col;
    const double *val;
    const double *b;
    double *x;
    double *ws;  // 9 n: r, dinv, z, p0, p1, w, t0, t1, t2
    // the sliced-diagonal copy (8 offset slots per slice) when the matrix is
    // on that schedule, else null: the tile products read it
    const int32_t *soff;
    const uint64_t *smask;
    const double *sval;
    int32_t n;
    int32_t U;
};

struct FState {
    double c[FDEG + 1];
    double lmax;
    double rho, delta, alpha, beta;
    double res, ref, best_res;
    int32_t its, fcg_its, best_its, status;
    int32_t flag, mode, restart, reason;
    int32_t zero_x, pad;
};

struct FPlan {
    const FSys *sys;                      // [nsys]
    const int32_t *tile_sys, *tile_row0;  // [ntiles]
    const int32_t *sys_tile0;             // [nsys + 1]
    const int32_t *sys_slice0;            // [nsys + 1]: first global 64-row slice of each system
    FState *st;                           // [nsys]
    double *part;                         // [4][nslices]: per 64-row slice, local slice l of system s at sys_slice0[s] + l
    unsigned *running;                    // [0]: systems still running; [2..3]: their rows (64-bit)
    int32_t nsys, ntiles, tiles_per_block;
    int32_t nslices;                      // sys_slice0[nsys]
    int32_t tile_rows;                    // rows per tile (a multiple of FT)
    int32_t maxit, stall_min, fallback;
    double rtol, stall_frac;
    int32_t force_jacobi;  // feature runs: every system in Jacobi mode from the start
    int32_t hist_cap;      // > 0: alpha, beta of the first hist_cap iterations
    double *hist;          // [nsys][2][hist_cap]
};

// Rows of the systems still running, kept beside the count.
__device__ __forceinline__ unsigned long long *running_rows(const FPlan &P) {
    return reinterpret_cast<unsigned long long *>(P.running + 2);
}

// The local slices [sl0, sl1) of tile t (of a system of n rows).
__device__ __forceinline__ void ftile_slices(const FPlan &P, int t, int n, int *sl0, int *sl1) {
    const int r0 = P.tile_row0[t];
    *sl0 = r0 >> 6;
    *sl1 = min((n + 63) >> 6, (r0 + P.tile_rows) >> 6);
}

// Runs body(t) for every tile t of this workgroup whose system passes
// keep(state).  Workgroup lb (its XCD-aware index) owns tiles lb, lb + G,
// lb + 2G, ...: the tiles of one system are spread over the grid, so the few
// systems still running at the end are worked on side by side.  Tiles are
// screened FT at a time -- each thread tests
// one tile, the survivors are compacted in LDS -- so a tail of stopped
// systems costs one round of loads per FT tiles, not a dependent chain per
// tile.  Each tile writes only its own outputs, so the order in which the
// survivors run does not change any result.
template <typename Keep, typename Body>
__device__ __forceinline__ void for_active_tiles(const FPlan &P, Keep keep, Body body) {
    const int lb = dev::xcd_block(blockIdx.x, gridDim.x), G = gridDim.x;
    __shared__ int list[FT];
    __shared__ int cnt;
    for (int base = 0; lb + base * G < P.ntiles; base += FT) {
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

// sum_k a_k u(col_k) over row i's entries; rows of up to 8 entries issue all
// gathers first (padded slots gather the row's own entry and are not added)
template <typename F>
__device__ __forceinline__ double frow(const dev::glob_t<int32_t> *col, const dev::glob_t<double> *val, int s, int e,
                                       int row, F u) {
    const int len = e - s;
    double sum = 0.0;
    if (len <= 8) {
        int jj[8];
        double aa[8], uj[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const bool in = q < len;
            jj[q] = in ? col[s + q] : row;
            aa[q] = in ? val[s + q] : 0.0;
        }
#pragma unroll
        for (int q = 0; q < 8; ++q) uj[q] = u(jj[q]);
#pragma unroll
        for (int q = 0; q < 8; ++q)
            if (q < len) sum = fma(aa[q], uj[q], sum);
    } else {
        for (int k = s; k < e; ++k) sum = fma(val[k], u(col[k]), sum);
    }
    return sum;
}

// Threads of the per-system kernels of the iteration (one workgroup per system).
constexpr int FSB = 256;

// The slice partials of system s (global slices sys_slice0[s] ..
// sys_slice0[s+1] of rows slot0.. of P.part), added in a fixed order (thread
// l takes slices l, l + FSB, ..., then the workgroup tree; one FSB-thread
// workgroup); the same sums whatever the tile size.  Result in thread 0.
template <int NV>
__device__ __forceinline__ void fsys_sum(const FPlan &P, int s, int slot0, double (&v)[NV]) {
    __shared__ double lds[NV * (FSB / 64)];
#pragma unroll
    for (int k = 0; k < NV; ++k) v[k] = 0.0;
    const int ge = P.sys_slice0[s + 1];
    const double *part = P.part + (size_t)slot0 * P.nslices;
    int g = P.sys_slice0[s] + (int)threadIdx.x;
    // eight of a thread's partials loaded before they are added (a large
    // system has thousands of slices); the same order of addition
    constexpr int UA = 8;
    for (; g + (UA - 1) * FSB < ge; g += UA * FSB) {
        double t[UA][NV];
#pragma unroll
        for (int u = 0; u < UA; ++u)
#pragma unroll
            for (int k = 0; k < NV; ++k) t[u][k] = part[(size_t)k * P.nslices + g + u * FSB];
#pragma unroll
        for (int u = 0; u < UA; ++u)
#pragma unroll
            for (int k = 0; k < NV; ++k) v[k] += t[u][k];
    }
    for (; g < ge; g += FSB) {
#pragma unroll
        for (int k = 0; k < NV; ++k) v[k] += part[(size_t)k * P.nslices + g];
    }
    dev::block_sum<FSB, NV>(v, lds);
}

// Per-tile partials (the feature passes): tiles of system s in index order.
template <int NV>
__device__ __forceinline__ void fsys_sum_tiles(const FPlan &P, int s, const double *part, double (&v)[NV]) {
    __shared__ double lds[NV];
#pragma unroll
    for (int k = 0; k < NV; ++k) v[k] = 0.0;
    for (int t = P.sys_tile0[s] + (int)threadIdx.x; t < P.sys_tile0[s + 1]; t += 64) {
#pragma unroll
        for (int k = 0; k < NV; ++k) v[k] += part[(size_t)k * P.ntiles + t];
    }
    dev::block_sum<64, NV>(v, lds);
}

// The calling wavefront's sums over its 64 rows (local slice sl of system s)
// as that slice's partials; lane 0 stores.  No workgroup barrier.
template <int NV>
__device__ __forceinline__ void ftile_store(const FPlan &P, int s, int sl, int slot0, double (&v)[NV]) {
#pragma unroll
    for (int k = 0; k < NV; ++k) v[k] = dev::wave_sum(v[k]);
    if ((threadIdx.x & 63) == 0) {
        const int g = P.sys_slice0[s] + sl;
#pragma unroll
        for (int k = 0; k < NV; ++k) P.part[(size_t)(slot0 + k) * P.nslices + g] = v[k];
    }
}

__device__ double fpoly_at(const double *c, double t, double lmax) {  // Clenshaw at one point
    const double y = 2.0 * t / lmax - 1.0;
    double b1 = 0.0, b2 = 0.0;
    for (int j = FDEG; j >= 1; --j) {
        const double b0 = c[j] + 2.0 * y * b1 - b2;
        b2 = b1;
        b1 = b0;
    }
    return c[0] + y * b1 - b2;
}

// Stops system s (thread 0 of its workgroup) with status, adding the fallback
// bits when it runs in Jacobi mode.
__device__ void fstop(const FPlan &P, FState *q, int status) {
    if (q->mode == MODE_JACOBI) status |= APCG_SOLVE_FALLBACK | q->reason;
    q->status = status;
    q->flag = 1;
    atomicSub(P.running, 1u);
    atomicAdd(running_rows(P), 0ull - (unsigned long long)P.sys[q - P.st].n);
}

// Hands system s over to Jacobi mode (reason: the failed test), or stops it
// when that is not possible.
__device__ void fswitch(const FPlan &P, FState *q, int reason) {
    if (q->mode == MODE_FLEX && P.fallback) {
        q->mode = MODE_JACOBI;
        q->reason = reason;
        q->restart = 1;
    } else {
        fstop(P, q, reason);
    }
}

__global__ __launch_bounds__(FT) void k_bf_init(FPlan P, int x0_zero) {
    const int tb0 = dev::xcd_block(blockIdx.x, gridDim.x), tstep = gridDim.x;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    for (int t = tb0; t < P.ntiles; t += tstep) {
      const int sys = P.tile_sys[t];
      const FSys S = P.sys[sys];
      int sl0, sl1;
      ftile_slices(P, t, S.n, &sl0, &sl1);
      for (int sl = sl0 + wave; sl < sl1; sl += FSW) {
        const int i = sl * 64 + lane;
        double v[3] = {0.0, 0.0, 0.0};  // ||b||^2, ||r||^2, bad diagonals
        if (i < S.n) {
            const int64_t n = S.n;
            double d = 0.0, ax = 0.0;
            bool found = false;
            for (int k = S.rowptr[i]; k < S.rowptr[i + 1]; ++k) {
                const int j = S.col[k];
                if (j == i) {
                    d = S.val[k];
                    found = true;
                }
                if (!x0_zero) ax = fma(S.val[k], S.x[j], ax);
            }
            const bool ok = found && d > 0.0;
            const double bi = S.b[i], ri = x0_zero ? bi : bi - ax;
            S.ws[i] = ri;
            S.ws[n + i] = ok ? 1.0 / d : 0.0;
            S.ws[3 * n + i] = 0.0;  // both direction buffers: the first beta is 0
            S.ws[4 * n + i] = 0.0;
            if (x0_zero) S.x[i] = 0.0;
            v[0] = bi * bi;
            v[1] = ri * ri;
            v[2] = ok ? 0.0 : 1.0;
        }
        ftile_store<3>(P, sys, sl, 0, v);
      }
    }
}

__global__ __launch_bounds__(FSB) void k_bf_init_final(FPlan P, const float *coef, const double *lmax) {
    const int s = blockIdx.x;
    double v[3];
    fsys_sum<3>(P, s, 0, v);
    __shared__ double cc[FDEG + 1];
    __shared__ int bad_point;
    const bool jac = P.force_jacobi != 0;
    if (threadIdx.x <= FDEG) cc[threadIdx.x] = jac ? (threadIdx.x == 0 ? 1.0 : 0.0)
                                                   : (double)coef[(size_t)s * (FDEG + 1) + threadIdx.x];
    if (threadIdx.x == 0) bad_point = 0;
    __syncthreads();
    const double lm = jac ? 1.0 : lmax[s];
    if (!jac)
        for (int q = threadIdx.x; q < 1024; q += FSB)
            if (!(fpoly_at(cc, lm * q / 1023.0, lm) > 0.0)) atomicOr(&bad_point, 1);
    __syncthreads();
    if (threadIdx.x != 0) return;
    FState q;
    for (int j = 0; j <= FDEG; ++j) q.c[j] = cc[j];
    q.lmax = lm;
    q.rho = q.delta = q.alpha = q.beta = 0.0;
    q.ref = sqrt(v[0]);
    q.res = sqrt(v[1]);
    q.best_res = q.res;
    q.its = q.fcg_its = q.best_its = 0;
    q.mode = MODE_FLEX;
    q.restart = 1;  // the first application of the preconditioner
    q.reason = 0;
    q.zero_x = 0;
    q.pad = 0;
    int status = 0;
    if (v[2] > 0.0) status = APCG_SOLVE_SETUP_ERROR;
    else if (q.ref == 0.0) {
        status = APCG_SOLVE_CONVERGED;
        q.zero_x = 1;
        q.res = 0.0;
    } else if (!isfinite(q.res) || !isfinite(q.ref)) status = APCG_SOLVE_NAN;
    else if (q.res <= P.rtol * q.ref) status = APCG_SOLVE_CONVERGED;
    else if (P.maxit <= 0) status = APCG_SOLVE_MAXIT;
    q.status = status;
    q.flag = status != 0;
    if (!q.flag && (bad_point || !(lm > 0.0) || !isfinite(lm))) {
        // the preconditioner would not be SPD
        if (P.fallback) {
            q.mode = MODE_JACOBI;
            q.reason = APCG_SOLVE_BREAKDOWN_RZ;
        } else {
            q.status = APCG_SOLVE_BREAKDOWN_RZ;
            q.flag = 1;
        }
    }
    if (jac) q.mode = MODE_JACOBI;  // reason 0: a plain Jacobi-PCG run
    P.st[s] = q;
    if (!q.flag) {
        atomicAdd(P.running, 1u);
        atomicAdd(running_rows(P), (unsigned long long)P.sys[s].n);
    }
}

__global__ __launch_bounds__(FT) void k_bf_zero_x(FPlan P) {
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    for_active_tiles(P, [](const FState &q) { return q.zero_x != 0; }, [&](int t) {
        const FSys S = P.sys[P.tile_sys[t]];
        int sl0, sl1;
        ftile_slices(P, t, S.n, &sl0, &sl1);
        for (int sl = sl0 + wave; sl < sl1; sl += FSW) {
            const int i = sl * 64 + lane;
            if (i < S.n) S.x[i] = 0.0;
        }
    });
}

// UC: sliced-diagonal slots walked per row (>= every such system's U).
template <int UC>
__global__ __launch_bounds__(FT) void k_bf_product(FPlan P, int parity) {
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    for_active_tiles(P, [](const FState &q) { return !q.flag && !q.restart; }, [&](int t) {
        const int s = P.tile_sys[t];
        const FState *q = P.st + s;
        const double beta = q->beta;
        const FSys S = P.sys[s];
        const int64_t n = S.n;
        const auto *z = dev::glb(S.ws + 2 * n);
        const auto *pold = dev::glb(S.ws + (3 + ((parity + 1) & 1)) * n);
        auto *pnew = dev::glb(S.ws + (3 + (parity & 1)) * n);
        auto *w = dev::glb(S.ws + 5 * n);
        int sl0, sl1;
        ftile_slices(P, t, S.n, &sl0, &sl1);
        auto u = [&](int j) { return fma(beta, pold[j], z[j]); };
        auto finish = [&](int sl, int i, int rc, double sum) {
            const double pi = fma(beta, pold[rc], z[rc]);
            double v[1] = {0.0};
            if (i < n) {
                pnew[i] = pi;
                w[i] = sum;
                v[0] = pi * sum;
            }
            ftile_store<1>(P, s, sl, 0, v);
        };
        if (S.sval) {  // the next slice's offsets and values loaded during the current gathers
            dev::sdia_slices<UC>(S.soff, S.smask, S.sval, S.U, n, sl0 + wave, sl1, FSW, u, finish);
            return;
        }
        for (int sl = sl0 + wave; sl < sl1; sl += FSW) {
            const int i = sl * 64 + lane;
            const int rc = i < n ? i : (int)n - 1;
            const auto *rp = dev::glb(S.rowptr);
            const double sum = i < n ? frow(dev::glb(S.col), dev::glb(S.val), rp[i], rp[i + 1], i, u) : 0.0;
            finish(sl, i, rc, sum);
        }
    });
}

__global__ __launch_bounds__(FSB) void k_bf_alpha(FPlan P) {
    const int s = blockIdx.x;
    FState *q = P.st + s;
    if (q->flag || q->restart) return;
    double v[1];
    fsys_sum<1>(P, s, 0, v);
    if (threadIdx.x != 0) return;
    const double delta = v[0];
    q->delta = delta;
    if (!(delta > 0.0)) {
        if (!isfinite(delta)) fstop(P, q, APCG_SOLVE_NAN);
        else fswitch(P, q, APCG_SOLVE_BREAKDOWN_PAP);
    } else {
        q->alpha = q->rho / delta;
        if (q->its < P.hist_cap) P.hist[(size_t)s * 2 * P.hist_cap + q->its] = q->alpha;
    }
}

__global__ __launch_bounds__(FT) void k_bf_update(FPlan P, int parity) {
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    for_active_tiles(P, [](const FState &q) { return !q.flag && !q.restart; }, [&](int t) {
        const int s = P.tile_sys[t];
        const FState *q = P.st + s;
        const double alpha = q->alpha;
        const FSys S = P.sys[s];
        const int64_t n = S.n;
        auto *r = dev::glb(S.ws);
        const auto *p = dev::glb(S.ws + (3 + (parity & 1)) * n);
        const auto *w = dev::glb(S.ws + 5 * n);
        auto *x = dev::glb(S.x);
        int sl0, sl1;
        ftile_slices(P, t, S.n, &sl0, &sl1);
        // the wavefront's slices in groups of UN whose loads are all issued
        // before the group's arithmetic and stores (per-slice sums unchanged)
        constexpr int UN = 4;
        for (int sb = sl0 + wave; sb < sl1; sb += UN * FSW) {
            double xs[UN], rs[UN], ps[UN], ws[UN];
#pragma unroll
            for (int u = 0; u < UN; ++u) {
                const int i = (sb + u * FSW) * 64 + lane;
                const int ic = (sb + u * FSW < sl1 && i < S.n) ? i : 0;
                xs[u] = x[ic];
                rs[u] = r[ic];
                ps[u] = p[ic];
                ws[u] = w[ic];
            }
#pragma unroll
            for (int u = 0; u < UN; ++u) {
                const int sl = sb + u * FSW;
                if (sl >= sl1) break;
                const int i = sl * 64 + lane;
                double v[1] = {0.0};
                if (i < S.n) {
                    x[i] = fma(alpha, ps[u], xs[u]);
                    const double ri = fma(-alpha, ws[u], rs[u]);
                    r[i] = ri;
                    v[0] = ri * ri;
                }
                ftile_store<1>(P, s, sl, 1, v);
            }
        }
    });
}

__global__ __launch_bounds__(FSB) void k_bf_check(FPlan P) {
    const int s = blockIdx.x;
    FState *q = P.st + s;
    if (q->flag || q->restart) return;
    double v[1];
    fsys_sum<1>(P, s, 1, v);
    if (threadIdx.x != 0) return;
    const double res = sqrt(v[0]);
    const int its = q->its + 1;
    q->its = its;
    q->res = res;
    if (q->mode == MODE_FLEX) q->fcg_its = its;
    if (!isfinite(res)) {
        fstop(P, q, APCG_SOLVE_NAN);
        return;
    }
    if (res <= P.rtol * q->ref) {
        fstop(P, q, APCG_SOLVE_CONVERGED);
        return;
    }
    if (q->mode == MODE_FLEX) {
        if (res < q->best_res) {
            q->best_res = res;
            q->best_its = its;
        } else {
            double win = P.stall_frac * (double)its;
            if (win < (double)P.stall_min) win = (double)P.stall_min;
            if ((double)(its - q->best_its) >= win) {
                fswitch(P, q, APCG_SOLVE_STALL);
                if (q->flag) return;
            }
        }
    }
    if (its >= P.maxit) fstop(P, q, APCG_SOLVE_MAXIT);
}

// One Clenshaw step of system s's polynomial.  stage 0: b_7 = c_7 v + 2 c_8 Y v;
// stage 1: b_j = c_j v + 2 Y b_{j+1} - b_{j+2}; stage 2: z = c_0 v + Y b_1 - b_2
// and the partials of r.z, z.w (Jacobi mode: z = v).  Y = (2/lmax) D^-1 A - I,
// v = D^-1 r; b_8 = c_8 v is formed where it is needed.
template <int UC>
__global__ __launch_bounds__(FT) void k_bf_cheb(FPlan P, int j, int stage, int o_b1, int o_b2, int o_out) {
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    for_active_tiles(P, [stage](const FState &q) { return !q.flag && (stage == 2 || q.mode != MODE_JACOBI); },
                     [&](int t) {
        const int s = P.tile_sys[t];
        const FState *q = P.st + s;
        const bool jac = q->mode == MODE_JACOBI;
        const FSys S = P.sys[s];
        const int64_t n = S.n;
        const auto *r = dev::glb(S.ws), *dinv = dev::glb(S.ws + n), *w = dev::glb(S.ws + 5 * n);
        const auto *bj1 = o_b1 >= 0 ? dev::glb(S.ws + (6 + o_b1) * n) : nullptr;
        const auto *bj2 = o_b2 >= 0 ? dev::glb(S.ws + (6 + o_b2) * n) : nullptr;
        auto *out = dev::glb(o_out >= 0 ? S.ws + (6 + o_out) * n : S.ws + 2 * n);
        const double s2 = 2.0 / q->lmax, cj = q->c[j], cd = q->c[FDEG];
        int sl0, sl1;
        ftile_slices(P, t, S.n, &sl0, &sl1);
        // the step once row i's sum of A u is known (au; unused in Jacobi mode).
        // Inlined at two call sites: contraction into FMAs is off so that
        // both compile to the same operations and the CSR and sliced-diagonal
        // reads give the same bits.
        auto finish = [&](int sl, int i, double au) {
#pragma clang fp contract(off)
            double v[2] = {0.0, 0.0};
            if (i < n) {
                const double vi = dinv[i] * r[i];
                double res;
                if (jac) {
                    res = vi;
                } else if (stage == 0) {
                    res = fma(2.0 * cd, s2 * dinv[i] * au - vi, cj * vi);
                } else {
                    const double yu = s2 * dinv[i] * au - bj1[i];
                    const double b2v = bj2 ? bj2[i] : cd * vi;
                    res = stage == 1 ? fma(2.0, yu, cj * vi) - b2v : cj * vi + yu - b2v;
                }
                out[i] = res;
                if (stage == 2) {
                    v[0] = r[i] * res;
                    v[1] = res * w[i];
                }
            }
            if (stage == 2) ftile_store<2>(P, s, sl, 2, v);
        };
        auto u0 = [&](int k) { return dinv[k] * r[k]; };
        auto u1 = [&](int k) { return bj1[k]; };
        if (!jac && S.sval) {  // the next slice's offsets and values loaded during the current gathers
            auto f = [&](int sl, int i, int, double au) { finish(sl, i, au); };
            if (stage == 0) dev::sdia_slices<UC>(S.soff, S.smask, S.sval, S.U, n, sl0 + wave, sl1, FSW, u0, f);
            else dev::sdia_slices<UC>(S.soff, S.smask, S.sval, S.U, n, sl0 + wave, sl1, FSW, u1, f);
            return;
        }
        for (int sl = sl0 + wave; sl < sl1; sl += FSW) {
            const int i = sl * 64 + lane;
            double au = 0.0;
            if (!jac && i < n)
                au = stage == 0 ? frow(dev::glb(S.col), dev::glb(S.val), dev::glb(S.rowptr)[i],
                                       dev::glb(S.rowptr)[i + 1], i, u0)
                                : frow(dev::glb(S.col), dev::glb(S.val), dev::glb(S.rowptr)[i],
                                       dev::glb(S.rowptr)[i + 1], i, u1);
            finish(sl, i, au);
        }
    });
}

__global__ __launch_bounds__(FSB) void k_bf_beta(FPlan P) {
    const int s = blockIdx.x;
    FState *q = P.st + s;
    if (q->flag) return;
    double v[2];
    fsys_sum<2>(P, s, 2, v);
    if (threadIdx.x != 0) return;
    const double rz = v[0], zw = v[1];
    if (q->restart) {  // a fresh recurrence from the current x
        if (!isfinite(rz)) fstop(P, q, APCG_SOLVE_NAN);
        else if (!(rz > 0.0)) fswitch(P, q, APCG_SOLVE_BREAKDOWN_RZ);  // stays in restart when switching
        else {
            q->rho = rz;
            q->beta = 0.0;
            q->restart = 0;
        }
        return;
    }
    if (!isfinite(rz) || !isfinite(zw)) fstop(P, q, APCG_SOLVE_NAN);
    else if (!(rz > 0.0)) fswitch(P, q, APCG_SOLVE_BREAKDOWN_RZ);
    else {
        q->beta = q->mode == MODE_FLEX ? -zw / q->delta : rz / q->rho;
        q->rho = rz;
        if (q->its - 1 < P.hist_cap) P.hist[(size_t)s * 2 * P.hist_cap + P.hist_cap + q->its - 1] = q->beta;
    }
}

// ---- batched features (the learned preconditioner's inputs) -------------
// Row statistics per tile -> fpart[k][t], k < 7 (dev::RowStats order).
__global__ __launch_bounds__(FT) void k_bf_rows(FPlan P, double *fpart) {
    const int tb0 = dev::xcd_block(blockIdx.x, gridDim.x), tstep = gridDim.x;
    __shared__ double sh[7][FT];
    for (int t = tb0; t < P.ntiles; t += tstep) {
        const FSys S = P.sys[P.tile_sys[t]];
        const int r0 = P.tile_row0[t], r1 = min(S.n, r0 + P.tile_rows);
        dev::RowStats a;
        for (int i = r0 + (int)threadIdx.x; i < r1; i += FT) dev::row_stats_add(a, S.rowptr, S.col, S.val, i);
        dev::row_stats_block<FT>(a, sh);
        if (threadIdx.x == 0)
            for (int k = 0; k < 7; ++k) fpart[(size_t)k * P.ntiles + t] = a.v[k];
        __syncthreads();
    }
}

// Per system (64 threads): thread l merges tiles l, l + 64, ... of the
// system, then the fixed tree -> fstats[s][0..6], fstats[s][7] = mean ln d.
__global__ __launch_bounds__(64) void k_bf_rows_final(FPlan P, const double *fpart, double *fstats) {
    const int s = blockIdx.x;
    dev::RowStats m;
    for (int t = P.sys_tile0[s] + (int)threadIdx.x; t < P.sys_tile0[s + 1]; t += 64) {
        double b[7];
        for (int k = 0; k < 7; ++k) b[k] = fpart[(size_t)k * P.ntiles + t];
        dev::row_stats_merge(m, b);
    }
    __shared__ double sh[7][64];
    dev::row_stats_block<64>(m, sh);
    if (threadIdx.x != 0) return;
    for (int k = 0; k < 7; ++k) fstats[8 * s + k] = m.v[k];
    const int n = P.sys[s].n;
    fstats[8 * s + 7] = n > 0 ? m.v[4] / (double)n : 0.0;
}

// sum (ln d_i - mean)^2 per tile -> fpart[7][t].
__global__ __launch_bounds__(FT) void k_bf_rows2(FPlan P, const double *fstats, double *fpart) {
    const int tb0 = dev::xcd_block(blockIdx.x, gridDim.x), tstep = gridDim.x;
    __shared__ double lds[FT / 64];
    for (int t = tb0; t < P.ntiles; t += tstep) {
        const int s = P.tile_sys[t];
        const FSys S = P.sys[s];
        const int r0 = P.tile_row0[t], r1 = min(S.n, r0 + P.tile_rows);
        double v[1] = {0.0};
        for (int i = r0 + (int)threadIdx.x; i < r1; i += FT) {
            const double e = dev::row_logdiag(S.rowptr, S.col, S.val, i) - fstats[8 * s + 7];
            v[0] = fma(e, e, v[0]);
        }
        dev::block_sum<FT, 1>(v, lds);
        if (threadIdx.x == 0) fpart[(size_t)7 * P.ntiles + t] = v[0];
        __syncthreads();
    }
}

// Per system: Ritz values of its recorded run (thread i < m: the i-th
// smallest), then the 16 features and lmax.  A system the run did not
// iterate on (b = 0) takes lmax as its only Ritz value.
__global__ __launch_bounds__(64) void k_bf_feat(FPlan P, const double *fpart, const double *fstats, float *feat,
                                                double *lmax_out) {
    const int s = blockIdx.x;
    const FState q = P.st[s];
    const double *al = P.hist + (size_t)s * 2 * P.hist_cap, *be = al + P.hist_cap;
    int m = q.its < P.hist_cap ? q.its : P.hist_cap;
    if (m > 16) m = 16;
    const double *st = fstats + 8 * s;
    __shared__ double th[16], td[16], te2[16];
    dev::ritz_values(al, be, m, td, te2, th);
    double vs[1];
    fsys_sum_tiles<1>(P, s, fpart + (size_t)7 * P.ntiles, vs);  // squared deviations over the tiles, fixed order
    __syncthreads();
    if (threadIdx.x != 0) return;
    if (m < 1) {
        th[0] = st[1];
        m = 1;
    }
    const double var = vs[0];
    const FSys S = P.sys[s];
    const double relres = q.ref > 0.0 ? q.res / q.ref : 1.0;
    dev::feature_vector(st, var, th, m, relres, S.n, (int64_t)S.rowptr[S.n], feat + (size_t)16 * s);
    lmax_out[s] = st[1];
}

__global__ void k_bf_finish(FPlan P, apcg_solve_info *info) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= P.nsys) return;
    const FState q = P.st[s];
    int status = q.status;
    if (!status) status = APCG_SOLVE_MAXIT | (q.mode == MODE_JACOBI ? APCG_SOLVE_FALLBACK | q.reason : 0);
    info[s].iterations = q.its;
    info[s].status = status;
    info[s].fcg_iterations = q.fcg_its;
    info[s].half_steps = 0;
    info[s].res_norm = q.res;
    info[s].ref_norm = q.ref;
}

__global__ void k_bf_reset(unsigned *running) {
    if (threadIdx.x < 4) running[threadIdx.x] = 0u;  // the count and the 64-bit row total
}

uint64_t fnv(const void *p, size_t n, uint64_t h = 1469598103934665603ull) {
    const unsigned char *c = static_cast<const unsigned char *>(p);
    for (size_t i = 0; i < n; ++i) h = (h ^ c[i]) * 1099511628211ull;
    return h;
}

}  // namespace

struct BfCache {
    int device = 0;
    FSys *d_sys = nullptr;
    int32_t *d_tile_sys = nullptr, *d_tile_row0 = nullptr, *d_sys_tile0 = nullptr, *d_sys_slice0 = nullptr;
    FState *d_st = nullptr;
    double *d_part = nullptr;  // 4 * slices_cap (slice partials)
    double *d_ws = nullptr;
    unsigned *d_running = nullptr;
    int64_t sys_cap = 0, tiles_cap = 0, ws_cap = 0, slices_cap = 0;
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
    // feature runs
    double *d_xs = nullptr;     // scratch iterates, offsets as the workspace's
    double *d_hist = nullptr;   // [sys_cap][2][FEAT_STEPS]
    double *d_fpart = nullptr;  // [8][tiles_cap]
    double *d_fstats = nullptr; // [sys_cap][8]
    float *d_X = nullptr;       // [sys_cap][16] features (learned solve)
    float *d_C = nullptr;       // [sys_cap][9] coefficients (learned solve)
    double *d_L = nullptr;      // [sys_cap] lmax (learned solve)
    int64_t feat_sys_cap = 0, feat_tiles_cap = 0, xs_cap = 0;
};

static std::mutex g_bf_mu;
static std::vector<std::pair<uint64_t, BfCache *>> g_bf;

static BfCache *bf_cache(apcg_ctx c) {
    std::lock_guard<std::mutex> lk(g_bf_mu);
    for (auto &p : g_bf)
        if (p.first == c->id) return p.second;
    BfCache *b = new BfCache();
    b->device = c->device;
    g_bf.emplace_back(c->id, b);
    return b;
}

static void bf_free_features(BfCache &b) {
    hipFree(b.d_xs);
    hipFree(b.d_hist);
    hipFree(b.d_fpart);
    hipFree(b.d_fstats);
    hipFree(b.d_X);
    hipFree(b.d_C);
    hipFree(b.d_L);
}

static void bf_free_tail(BfCache &b) {
    if (b.exec_t) hipGraphExecDestroy(b.exec_t);
    if (b.graph_t) hipGraphDestroy(b.graph_t);
    hipFree(b.d_tile_sys_t);
    hipFree(b.d_tile_row0_t);
}

static void bf_free(BfCache &b) {
    if (b.exec) hipGraphExecDestroy(b.exec);
    if (b.graph) hipGraphDestroy(b.graph);
    hipFree(b.d_sys);
    hipFree(b.d_tile_sys);
    hipFree(b.d_tile_row0);
    hipFree(b.d_sys_tile0);
    hipFree(b.d_sys_slice0);
    hipFree(b.d_st);
    hipFree(b.d_part);
    hipFree(b.d_ws);
    hipFree(b.d_running);
}

void bfcg_cache_release(uint64_t ctx_id, int device) {
    BfCache *b = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_bf_mu);
        for (auto it = g_bf.begin(); it != g_bf.end(); ++it)
            if (it->first == ctx_id) {
                b = it->second;
                g_bf.erase(it);
                break;
            }
    }
    if (!b) return;
    hipSetDevice(device);
    bf_free(*b);
    bf_free_tail(*b);
    bf_free_features(*b);
    if (b->pinned) hipHostFree(b->pinned);
    delete b;
}

}  // namespace apcg

namespace apcg {

constexpr int FEAT_STEPS = 12;  // Jacobi-PCG steps of the feature run
// The tail plan takes over once the rows still running fill fewer than this
// many of the large tiles per compute unit: on the 1024-system mixed batch
// (2048-row tiles, a 256-row tail) 2 -> 8.95 s, 8 -> 8.77, 16 -> 8.71,
// 32 -> 8.68, 64 -> 8.67 s, against 8.97 s without the switch.
constexpr uint64_t kTailTilesPerCu = 32;

// What one run of the batched iteration computes.
struct BfRun {
    const float *coeffs = nullptr;   // [nsys][9]
    const double *lmax = nullptr;    // [nsys]
    int force_jacobi = 0;            // feature run: plain Jacobi-PCG for every system
    double *hist = nullptr;          // [nsys][2][hist_cap]
    int32_t hist_cap = 0;
};

// Enqueues one run of the batched iteration on ctx's stream.  hs: the
// systems (ws holds workspace offsets on entry); xs_base != nullptr: x of
// system i is xs_base + its workspace offset / 9 (the feature run's scratch).
static apcg_status bf_core(apcg_ctx ctx, BfCache *bc, int32_t nsys, std::vector<FSys> &hs, int64_t ws_total,
                           const std::vector<apcg_mat_s *> &refill, double rtol, int32_t maxit,
                           const apcg_solve_opts &opts, const apcg_fcg_opts &fo, const BfRun &run,
                           apcg_solve_info *d_info, FPlan *plan_out = nullptr, int *grid_out = nullptr) {
    const int dev = ctx->device;
    hipStream_t st = ctx->stream;
    for (apcg_mat_s *m : refill) {  // the sliced-diagonal values of the systems that read them
        apcg_status ps = prepare_sdia(m, st);
        if (ps) return ps;
    }
    const int32_t TR = batch_tile_rows(opts);
    std::vector<int32_t> tile_sys, tile_row0, sys_tile0(nsys + 1), sys_slice0(nsys + 1);
    int64_t nslices = 0;
    for (int32_t q = 0; q < nsys; ++q) {
        sys_tile0[q] = (int32_t)tile_sys.size();
        sys_slice0[q] = (int32_t)nslices;
        nslices += ((int64_t)hs[q].n + 63) / 64;
        for (int32_t r0 = 0; r0 < hs[q].n; r0 += TR) {
            tile_sys.push_back(q);
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
    const int32_t TRt = run.force_jacobi ? 0 : batch_tail_rows(opts);
    std::vector<int32_t> tile_sys_t, tile_row0_t;
    if (TRt > 0)
        for (int32_t q = 0; q < nsys; ++q)
            for (int32_t r0 = 0; r0 < hs[q].n; r0 += TRt) {
                tile_sys_t.push_back(q);
                tile_row0_t.push_back(r0);
            }
    const int32_t ntiles_t = (int32_t)tile_sys_t.size();
    const bool tail_plan = ntiles_t > 0;
    const int64_t ns_alloc = std::max<int64_t>(nslices, 1);
    const int32_t ntiles = (int32_t)tile_sys.size();
    if (ntiles == 0) {  // every system is empty: one dummy tile keeps the kernels well formed
        tile_sys.push_back(0);
        tile_row0.push_back(0);
    }
    const int32_t nt_alloc = std::max<int32_t>(ntiles, 1);
    APCG_HIP(hipSetDevice(dev));
    const int64_t ws_need = std::max<int64_t>(ws_total, 64);
    if (bc->sys_cap < nsys || bc->tiles_cap < nt_alloc || bc->ws_cap < ws_need || bc->slices_cap < ns_alloc) {
        EventRef ev = event_get(dev);
        if (!ev) return set_error(APCG_ERR_HIP, "event creation failed");
        APCG_HIP(hipEventRecord(ev->e, st));
        BfCache old = *bc;
        defer_release({ev}, [old]() mutable {
            hipSetDevice(old.device);
            bf_free(old);
        });
        bc->exec = nullptr;
        bc->graph = nullptr;
        bc->graph_hash = 0;
        bc->hash = 0;
        bc->sys_cap = std::max<int64_t>(nsys, bc->sys_cap);
        bc->tiles_cap = std::max<int64_t>(nt_alloc, bc->tiles_cap);
        bc->slices_cap = std::max<int64_t>(ns_alloc, bc->slices_cap);
        bc->ws_cap = std::max<int64_t>(ws_need, bc->ws_cap);
        APCG_HIP(hipMalloc((void **)&bc->d_sys, sizeof(FSys) * bc->sys_cap));
        APCG_HIP(hipMalloc((void **)&bc->d_st, sizeof(FState) * bc->sys_cap));
        APCG_HIP(hipMalloc((void **)&bc->d_sys_tile0, sizeof(int32_t) * (bc->sys_cap + 1)));
        APCG_HIP(hipMalloc((void **)&bc->d_sys_slice0, sizeof(int32_t) * (bc->sys_cap + 1)));
        APCG_HIP(hipMalloc((void **)&bc->d_tile_sys, sizeof(int32_t) * bc->tiles_cap));
        APCG_HIP(hipMalloc((void **)&bc->d_tile_row0, sizeof(int32_t) * bc->tiles_cap));
        APCG_HIP(hipMalloc((void **)&bc->d_part, sizeof(double) * 4 * bc->slices_cap));
        APCG_HIP(hipMalloc((void **)&bc->d_ws, sizeof(double) * bc->ws_cap));
        APCG_HIP(hipMalloc((void **)&bc->d_running, 256));
    }
    if (!bc->pinned)
        APCG_HIP(hipHostMalloc((void **)&bc->pinned, sizeof(int32_t) * 4 * kMaxLookahead, hipHostMallocDefault));
    for (int32_t i = 0; i < nsys; ++i) hs[i].ws = bc->d_ws + reinterpret_cast<int64_t>(hs[i].ws);
    uint64_t h = fnv(hs.data(), sizeof(FSys) * nsys);
    h = fnv(tile_sys.data(), sizeof(int32_t) * tile_sys.size(), h);
    h = fnv(tile_row0.data(), sizeof(int32_t) * tile_row0.size(), h);
    h = fnv(sys_tile0.data(), sizeof(int32_t) * sys_tile0.size(), h);
    h = fnv(sys_slice0.data(), sizeof(int32_t) * sys_slice0.size(), h);
    if (h != bc->hash) {
        g_counters.h2d_copies += 5;
        APCG_HIP(hipMemcpyAsync(bc->d_sys_slice0, sys_slice0.data(), sizeof(int32_t) * sys_slice0.size(),
                                hipMemcpyHostToDevice, st));
        APCG_HIP(hipMemcpyAsync(bc->d_sys, hs.data(), sizeof(FSys) * nsys, hipMemcpyHostToDevice, st));
        APCG_HIP(hipMemcpyAsync(bc->d_tile_sys, tile_sys.data(), sizeof(int32_t) * tile_sys.size(),
                                hipMemcpyHostToDevice, st));
        APCG_HIP(hipMemcpyAsync(bc->d_tile_row0, tile_row0.data(), sizeof(int32_t) * tile_row0.size(),
                                hipMemcpyHostToDevice, st));
        APCG_HIP(hipMemcpyAsync(bc->d_sys_tile0, sys_tile0.data(), sizeof(int32_t) * sys_tile0.size(),
                                hipMemcpyHostToDevice, st));
        g_counters.host_syncs++;
        APCG_HIP(hipStreamSynchronize(st));  // the host tables are local
        bc->hash = h;
    }
    if (tail_plan) {
        if (bc->tiles_t_cap < ntiles_t) {
            EventRef ev = event_get(dev);
            if (!ev) return set_error(APCG_ERR_HIP, "event creation failed");
            APCG_HIP(hipEventRecord(ev->e, st));
            BfCache old = *bc;
            defer_release({ev}, [old]() mutable {
                hipSetDevice(old.device);
                bf_free_tail(old);
            });
            bc->exec_t = nullptr;
            bc->graph_t = nullptr;
            bc->graph_hash_t = 0;
            bc->hash_t = 0;
            bc->tiles_t_cap = ntiles_t;
            APCG_HIP(hipMalloc((void **)&bc->d_tile_sys_t, sizeof(int32_t) * bc->tiles_t_cap));
            APCG_HIP(hipMalloc((void **)&bc->d_tile_row0_t, sizeof(int32_t) * bc->tiles_t_cap));
        }
        uint64_t ht = fnv(tile_sys_t.data(), sizeof(int32_t) * tile_sys_t.size());
        ht = fnv(tile_row0_t.data(), sizeof(int32_t) * tile_row0_t.size(), ht);
        if (ht != bc->hash_t) {
            g_counters.h2d_copies += 2;
            APCG_HIP(hipMemcpyAsync(bc->d_tile_sys_t, tile_sys_t.data(), sizeof(int32_t) * tile_sys_t.size(),
                                    hipMemcpyHostToDevice, st));
            APCG_HIP(hipMemcpyAsync(bc->d_tile_row0_t, tile_row0_t.data(), sizeof(int32_t) * tile_row0_t.size(),
                                    hipMemcpyHostToDevice, st));
            g_counters.host_syncs++;
            APCG_HIP(hipStreamSynchronize(st));  // the host tables are local
            bc->hash_t = ht;
        }
        if (!bc->cus) APCG_HIP(hipDeviceGetAttribute(&bc->cus, hipDeviceAttributeMultiprocessorCount, dev));
    }
    FPlan P;
    P.sys = bc->d_sys;
    P.tile_sys = bc->d_tile_sys;
    P.tile_row0 = bc->d_tile_row0;
    P.sys_tile0 = bc->d_sys_tile0;
    P.sys_slice0 = bc->d_sys_slice0;
    P.st = bc->d_st;
    P.part = bc->d_part;
    P.running = bc->d_running;
    P.nsys = nsys;
    P.ntiles = ntiles;
    P.nslices = (int32_t)ns_alloc;
    P.tile_rows = TR;
    const int G = normalise_blocks(kMaxBlocks, std::max<int32_t>(ntiles, 1));  // few tiles per workgroup: more in flight
    P.tiles_per_block = std::max<int32_t>(1, (ntiles + G - 1) / G);
    P.maxit = maxit;
    if (plan_out) *plan_out = P;
    if (grid_out) *grid_out = G;
    P.stall_min = fo.stall_min;
    P.fallback = fo.fallback ? 1 : 0;
    P.rtol = rtol;
    P.stall_frac = fo.stall_frac;
    P.force_jacobi = run.force_jacobi;
    P.hist_cap = run.hist ? run.hist_cap : 0;
    P.hist = run.hist;
    FPlan Pt = P;
    int Gt = G;
    if (tail_plan) {
        Pt.tile_sys = bc->d_tile_sys_t;
        Pt.tile_row0 = bc->d_tile_row0_t;
        Pt.ntiles = ntiles_t;
        Pt.tile_rows = TRt;
        Gt = normalise_blocks(kMaxBlocks, ntiles_t);
        Pt.tiles_per_block = std::max<int32_t>(1, (ntiles_t + Gt - 1) / Gt);
    }
    // switch when the running rows fill fewer than kTailTilesPerCu large tiles per CU
    const uint64_t tail_rows = tail_plan ? kTailTilesPerCu * (uint64_t)bc->cus * (uint64_t)TR : 0;
    const int x0z = opts.x0_is_zero ? 1 : 0;
    apcg_status s;

    hipLaunchKernelGGL(k_bf_reset, dim3(1), dim3(64), 0, st, bc->d_running);
    APCG_CHECK_LAUNCH("k_bf_reset");
    hipLaunchKernelGGL(k_bf_init, dim3(G), dim3(FT), 0, st, P, x0z);
    APCG_CHECK_LAUNCH("k_bf_init");
    hipLaunchKernelGGL(k_bf_init_final, dim3(nsys), dim3(FSB), 0, st, P, run.coeffs, run.lmax);
    APCG_CHECK_LAUNCH("k_bf_init_final");
    if (!x0z) {
        hipLaunchKernelGGL(k_bf_zero_x, dim3(G), dim3(FT), 0, st, P);
        APCG_CHECK_LAUNCH("k_bf_zero_x");
    }
    int K = std::max(2, opts.iters_per_graph);
    if (K & 1) ++K;
    const int L = std::max(1, std::min(kMaxLookahead, opts.lookahead));
    int umax = 0;  // most sliced-diagonal slots of any system that reads them
    for (int32_t i = 0; i < nsys; ++i)
        if (hs[i].sval) umax = std::max<int>(umax, hs[i].U);
    const int uc = umax <= 5 ? 5 : umax <= 7 ? 7 : 8;
    void (*bf_product)(FPlan, int) = uc == 5 ? k_bf_product<5> : uc == 7 ? k_bf_product<7> : k_bf_product<8>;
    void (*bf_cheb)(FPlan, int, int, int, int, int) = uc == 5 ? k_bf_cheb<5> : uc == 7 ? k_bf_cheb<7> : k_bf_cheb<8>;
    // Clenshaw buffers t0..t2 round robin: b_j in t[j % 3]
    auto launch_iter = [&](int j, const FPlan &P, int G) -> apcg_status {
        hipLaunchKernelGGL(bf_product, dim3(G), dim3(FT), 0, st, P, j & 1);
        APCG_CHECK_LAUNCH("k_bf_product");
        hipLaunchKernelGGL(k_bf_alpha, dim3(nsys), dim3(FSB), 0, st, P);
        APCG_CHECK_LAUNCH("k_bf_alpha");
        hipLaunchKernelGGL(k_bf_update, dim3(G), dim3(FT), 0, st, P, j & 1);
        APCG_CHECK_LAUNCH("k_bf_update");
        hipLaunchKernelGGL(k_bf_check, dim3(nsys), dim3(FSB), 0, st, P);
        APCG_CHECK_LAUNCH("k_bf_check");
        for (int d = FDEG - 1; d >= 0; --d) {
            const int stage = d == FDEG - 1 ? 0 : (d == 0 ? 2 : 1);
            if (run.force_jacobi && stage != 2) continue;  // Jacobi mode: only z = D^-1 r
            const int ob1 = stage == 0 ? -1 : (d + 1) % 3;
            const int ob2 = (stage == 0 || d + 2 == FDEG) ? -1 : (d + 2) % 3;
            const int oout = stage == 2 ? -1 : d % 3;
            hipLaunchKernelGGL(bf_cheb, dim3(G), dim3(FT), 0, st, P, d, stage, ob1, ob2, oout);
            APCG_CHECK_LAUNCH("k_bf_cheb");
        }
        hipLaunchKernelGGL(k_bf_beta, dim3(nsys), dim3(FSB), 0, st, P);
        APCG_CHECK_LAUNCH("k_bf_beta");
        return APCG_SUCCESS;
    };
    // K iterations of plan Pc on grid Gc captured into one executable graph
    auto capture = [&](const FPlan &Pc, int Gc, hipGraph_t *gout, hipGraphExec_t *xout) -> apcg_status {
        APCG_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeRelaxed));
        apcg_status cs = APCG_SUCCESS;
        for (int j = 1; j <= K && cs == APCG_SUCCESS; ++j) cs = launch_iter(j, Pc, Gc);
        hipGraph_t g = nullptr;
        hipError_t e = hipStreamEndCapture(st, &g);
        if (cs) {
            if (g) hipGraphDestroy(g);
            return cs;
        }
        if (e != hipSuccess) return hip_error(e, "hipStreamEndCapture(batched fcg)");
        g_counters.kernel_launches -= (int64_t)(5 + FDEG) * K;
        e = hipGraphInstantiate(xout, g, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            hipGraphDestroy(g);
            return hip_error(e, "hipGraphInstantiate(batched fcg)");
        }
        *gout = g;
        return APCG_SUCCESS;
    };
    const bool graph = opts.mode == APCG_MODE_GRAPH && !run.force_jacobi;  // feature runs are short: no capture
    uint64_t gh = fnv(&h, sizeof h);
    const double prm[2] = {rtol, fo.stall_frac};
    const int iprm[8] = {K, maxit, G, nsys, fo.stall_min, P.fallback, P.tiles_per_block, uc};
    gh = fnv(prm, sizeof prm, gh);
    gh = fnv(iprm, sizeof iprm, gh);
    const void *ptrs[3] = {bc->d_st, bc->d_part, bc->d_running};
    gh = fnv(ptrs, sizeof ptrs, gh);
    if (maxit > 0) {
        if (graph && (!bc->exec || bc->graph_hash != gh)) {
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
            if ((s = capture(P, G, &bc->graph, &bc->exec))) return s;
            bc->graph_hash = gh;
        }
        // the tail plan's period, captured alike
        uint64_t ght = fnv(&bc->hash_t, sizeof bc->hash_t, gh);
        const int tprm[3] = {Gt, TRt, Pt.tiles_per_block};
        ght = fnv(tprm, sizeof tprm, ght);
        const void *tptrs[2] = {bc->d_tile_sys_t, bc->d_tile_row0_t};
        ght = fnv(tptrs, sizeof tptrs, ght);
        if (graph && tail_plan && (!bc->exec_t || bc->graph_hash_t != ght)) {
            if (bc->exec_t) {
                EventRef ev = event_get(dev);
                if (ev) hipEventRecord(ev->e, st);
                hipGraphExec_t oe = bc->exec_t;
                hipGraph_t og = bc->graph_t;
                defer_release({ev}, [oe, og, dev]() {
                    hipSetDevice(dev);
                    hipGraphExecDestroy(oe);
                    hipGraphDestroy(og);
                });
                bc->exec_t = nullptr;
                bc->graph_t = nullptr;
            }
            if ((s = capture(Pt, Gt, &bc->graph_t, &bc->exec_t))) return s;
            bc->graph_hash_t = ght;
        }
        // iteration slots: maxit counted iterations plus at most two
        // restarts per system (the first application and one switch)
        const int64_t periods = ((int64_t)maxit + 2 + K - 1) / K;
        bool tail = false;  // periods on the tail plan from here on
        for (int64_t g = 0; g < periods; ++g) {
            if (graph) {
                g_counters.graph_launches++;
                APCG_HIP(hipGraphLaunch(tail ? bc->exec_t : bc->exec, st));
            } else {
                for (int j = 1; j <= K; ++j)
                    if ((s = launch_iter(j, tail ? Pt : P, tail ? Gt : G))) return s;
            }
            const int slot = (int)(g % L);
            if (!bc->poll_ev[slot]) {
                bc->poll_ev[slot] = event_get(dev);
                if (!bc->poll_ev[slot]) return set_error(APCG_ERR_HIP, "event creation failed");
            }
            g_counters.d2h_copies++;
            APCG_HIP(hipMemcpyAsync(&bc->pinned[4 * slot], bc->d_running, 4 * sizeof(int32_t), hipMemcpyDeviceToHost,
                                    st));
            APCG_HIP(hipEventRecord(bc->poll_ev[slot]->e, st));
            if (g >= L - 1) {
                const int ps = (int)((g - (L - 1)) % L);
                g_counters.host_polls++;
                APCG_HIP(hipEventSynchronize(bc->poll_ev[ps]->e));
                if (bc->pinned[4 * ps] == 0) break;  // every system has stopped
                uint64_t rows;
                memcpy(&rows, &bc->pinned[4 * ps + 2], sizeof rows);
                if (tail_plan && !tail && rows < tail_rows) tail = true;
            }
        }
    }
    if (d_info) {
        hipLaunchKernelGGL(k_bf_finish, dim3((nsys + 63) / 64), dim3(64), 0, st, P, d_info);
        APCG_CHECK_LAUNCH("k_bf_finish");
    }
    return APCG_SUCCESS;
}

// Checks the systems and builds their descriptors (workspace offsets in ws).
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

static apcg_status bf_systems(apcg_ctx ctx, int32_t nsys, const apcg_mat *A, const apcg_vec *b, const apcg_vec *x,
                              std::vector<FSys> &hs, int64_t *ws_total, std::vector<apcg_mat_s *> &refill) {
    const int dev = ctx->device;
    hs.resize(nsys);
    int64_t tot = 0;
    for (int32_t i = 0; i < nsys; ++i) {
        if (!A[i] || !b[i] || (x && !x[i])) return set_error(APCG_ERR_INVALID_ARG, "NULL system handle");
        if (A[i]->device != dev || b[i]->device != dev || (x && x[i]->device != dev))
            return set_error(APCG_ERR_INVALID_ARG, "operands on different devices");
        if (b[i]->n != A[i]->n || (x && x[i]->n != A[i]->n))
            return set_error(APCG_ERR_INVALID_ARG, "dimension mismatch");
        if (x && (b[i] == x[i] || (b[i]->d == x[i]->d && A[i]->n > 0)))
            return set_error(APCG_ERR_INVALID_ARG, "b and x must not alias");
        const int64_t n = A[i]->n;
        hs[i] = FSys{A[i]->rowptr, A[i]->col, A[i]->val, b[i]->d, x ? x[i]->d : nullptr,
                     reinterpret_cast<double *>(tot), nullptr, nullptr, nullptr, (int32_t)n, 0};
        if (A[i]->cfg.schedule == APCG_SPMV_SDIA && A[i]->sdia_state == 1 && A[i]->sdia_mp == 8) {
            hs[i].soff = A[i]->sdia_off;
            hs[i].smask = A[i]->sdia_msk;
            hs[i].sval = A[i]->sdia_val;
            hs[i].U = A[i]->sdia_u;
            refill.push_back(A[i]);
        }
        tot += ((9 * n + 63) / 64) * 64;
    }
    if (x)
        if (apcg_status s = check_batch_ranges(nsys, b, x)) return s;
    *ws_total = tot;
    return APCG_SUCCESS;
}

static apcg_status bf_common_checks(apcg_ctx ctx, int32_t nsys, const void *A, const void *b) {
    if (!ctx || nsys < 1 || !A || !b) return set_error(APCG_ERR_INVALID_ARG, "NULL argument");
    if (ctx->type == APCG_STREAM_GLOBAL_BLOCKING && ctx->is_default_global)
        return set_error(APCG_ERR_INVALID_ARG, "pass a context created with apcg_ctx_create");
    return APCG_SUCCESS;
}

// Features of every system into feat[nsys][16] / lmax[nsys] (device), on
// ctx: one batched 12-step Jacobi-PCG run from x0 = 0 on scratch iterates
// with alpha/beta recorded, two passes of row statistics, the Ritz values.
static apcg_status bf_features(apcg_ctx ctx, BfCache *bc, int32_t nsys, const apcg_mat *A, const apcg_vec *b,
                               float *feat, double *lmax) {
    std::vector<FSys> hs;
    std::vector<apcg_mat_s *> refill;
    int64_t ws_total = 0;
    apcg_status s;
    if ((s = bf_systems(ctx, nsys, A, b, nullptr, hs, &ws_total, refill))) return s;
    const int dev = ctx->device;
    hipStream_t st = ctx->stream;
    APCG_HIP(hipSetDevice(dev));
    int64_t ntiles = 0;
    for (auto &f : hs) ntiles += (f.n + FT - 1) / FT;
    ntiles = std::max<int64_t>(ntiles, 1);
    const int64_t xs_need = std::max<int64_t>(ws_total / 9 + 64, 64);
    if (bc->feat_sys_cap < nsys || bc->feat_tiles_cap < ntiles || bc->xs_cap < xs_need) {
        EventRef ev = event_get(dev);
        if (!ev) return set_error(APCG_ERR_HIP, "event creation failed");
        APCG_HIP(hipEventRecord(ev->e, st));
        BfCache old = *bc;
        defer_release({ev}, [old]() mutable {
            hipSetDevice(old.device);
            bf_free_features(old);
        });
        bc->feat_sys_cap = std::max<int64_t>(nsys, bc->feat_sys_cap);
        bc->feat_tiles_cap = std::max<int64_t>(ntiles, bc->feat_tiles_cap);
        bc->xs_cap = std::max<int64_t>(xs_need, bc->xs_cap);
        APCG_HIP(hipMalloc((void **)&bc->d_xs, sizeof(double) * bc->xs_cap));
        APCG_HIP(hipMalloc((void **)&bc->d_hist, sizeof(double) * 2 * FEAT_STEPS * bc->feat_sys_cap));
        APCG_HIP(hipMalloc((void **)&bc->d_fpart, sizeof(double) * 8 * bc->feat_tiles_cap));
        APCG_HIP(hipMalloc((void **)&bc->d_fstats, sizeof(double) * 8 * bc->feat_sys_cap));
        APCG_HIP(hipMalloc((void **)&bc->d_X, sizeof(float) * 16 * bc->feat_sys_cap));
        APCG_HIP(hipMalloc((void **)&bc->d_C, sizeof(float) * 9 * bc->feat_sys_cap));
        APCG_HIP(hipMalloc((void **)&bc->d_L, sizeof(double) * bc->feat_sys_cap));
    }
    if (!feat) feat = bc->d_X;  // the learned solve keeps them in the cache
    if (!lmax) lmax = bc->d_L;
    // scratch iterates: the workspace offset / 9 keeps every system's range apart
    for (auto &f : hs) f.x = bc->d_xs + reinterpret_cast<int64_t>(f.ws) / 9;
    apcg_solve_opts o;
    apcg_solve_opts_default(&o);
    o.x0_is_zero = 1;
    o.mode = APCG_MODE_STREAM;
    o.iters_per_graph = FEAT_STEPS + 2;  // one period: the first application and the steps
    apcg_fcg_opts fo;
    apcg_fcg_opts_default(&fo);
    fo.fallback = 0;
    BfRun run;
    run.force_jacobi = 1;
    run.hist = bc->d_hist;
    run.hist_cap = FEAT_STEPS;
    FPlan P;
    int G = 0;
    if ((s = bf_core(ctx, bc, nsys, hs, ws_total, refill, 0.0, FEAT_STEPS, o, fo, run, nullptr, &P, &G))) return s;
    P.hist = bc->d_hist;
    P.hist_cap = FEAT_STEPS;
    hipLaunchKernelGGL(k_bf_rows, dim3(G), dim3(FT), 0, st, P, bc->d_fpart);
    APCG_CHECK_LAUNCH("k_bf_rows");
    hipLaunchKernelGGL(k_bf_rows_final, dim3(nsys), dim3(64), 0, st, P, (const double *)bc->d_fpart, bc->d_fstats);
    APCG_CHECK_LAUNCH("k_bf_rows_final");
    hipLaunchKernelGGL(k_bf_rows2, dim3(G), dim3(FT), 0, st, P, (const double *)bc->d_fstats, bc->d_fpart);
    APCG_CHECK_LAUNCH("k_bf_rows2");
    hipLaunchKernelGGL(k_bf_feat, dim3(nsys), dim3(64), 0, st, P, (const double *)bc->d_fpart,
                       (const double *)bc->d_fstats, feat, lmax);
    APCG_CHECK_LAUNCH("k_bf_feat");
    return APCG_SUCCESS;
}

}  // namespace apcg

using namespace apcg;

extern "C" apcg_status apcg_ksp_solve_batched_fcg_poly(apcg_ctx ctx, int32_t nsys, const apcg_mat *A,
                                                       const apcg_vec *b, const apcg_vec *x, double rtol,
                                                       int32_t maxit, const float *dev_coeffs,
                                                       const double *dev_lmax, const apcg_solve_opts *opts_in,
                                                       const apcg_fcg_opts *fopts_in, apcg_info info) {
    try {
        apcg_status s;
        if ((s = bf_common_checks(ctx, nsys, A, b))) return s;
        if (!x || !info || !dev_coeffs || !dev_lmax) return set_error(APCG_ERR_INVALID_ARG, "NULL argument");
        if (info->count < nsys || info->device != ctx->device)
            return set_error(APCG_ERR_INVALID_ARG, "info has fewer records than systems or another device");
        if (!(rtol >= 0.0) || !std::isfinite(rtol)) return set_error(APCG_ERR_INVALID_ARG, "rtol must be finite and >= 0");
        if (maxit < 0) return set_error(APCG_ERR_INVALID_ARG, "maxit must be >= 0");
        apcg_solve_opts opts;
        if (opts_in) opts = *opts_in;
        else apcg_solve_opts_default(&opts);
        apcg_fcg_opts fo;
        if (fopts_in) fo = *fopts_in;
        else apcg_fcg_opts_default(&fo);
        if (fo.stall_min < 1 || !(fo.stall_frac >= 0.0)) return set_error(APCG_ERR_INVALID_ARG, "bad stall window");
        if (!valid_batch_tail_rows(opts.batch_tail_tile_rows))
            return set_error(APCG_ERR_INVALID_ARG, "batch tail tile rows must be -1, 0 or a multiple of 256 in [256, 8192]");
        if (!valid_batch_tile_rows(opts.batch_tile_rows))
            return set_error(APCG_ERR_INVALID_ARG, "batch tile rows must be 0 or a multiple of 256 in [256, 8192]");
        std::vector<FSys> hs;
        std::vector<apcg_mat_s *> refill;
        int64_t ws_total = 0;
        if ((s = bf_systems(ctx, nsys, A, b, x, hs, &ws_total, refill))) return s;
        std::vector<Acc> acc;
        acc.reserve(3 * nsys + 1);
        for (int32_t i = 0; i < nsys; ++i) {
            acc.push_back({&x[i]->rec, ACC_RW});
            acc.push_back({&A[i]->rec, ACC_R});
            acc.push_back({&b[i]->rec, ACC_R});
        }
        acc.push_back({&info->rec, ACC_W});
        if ((s = op_begin(ctx, acc.data(), (int)acc.size()))) return s;
        BfRun run;
        run.coeffs = dev_coeffs;
        run.lmax = dev_lmax;
        if ((s = bf_core(ctx, bf_cache(ctx), nsys, hs, ws_total, refill, rtol, maxit, opts, fo, run, info->d))) return s;
        return op_end(ctx, acc.data(), (int)acc.size());
    } catch (const std::bad_alloc &) {
        return set_error(APCG_ERR_OUT_OF_MEMORY, "host allocation failed");
    }
}

extern "C" apcg_status apcg_pc_features_batched(apcg_ctx ctx, int32_t nsys, const apcg_mat *A, const apcg_vec *b,
                                                float *dev_feat, double *dev_lmax) {
    try {
        apcg_status s;
        if ((s = bf_common_checks(ctx, nsys, A, b))) return s;
        if (!dev_feat || !dev_lmax) return set_error(APCG_ERR_INVALID_ARG, "NULL argument");
        std::vector<Acc> acc;
        acc.reserve(2 * nsys);
        for (int32_t i = 0; i < nsys; ++i) {
            if (!A[i] || !b[i]) return set_error(APCG_ERR_INVALID_ARG, "NULL system handle");
            acc.push_back({&A[i]->rec, ACC_R});
            acc.push_back({&b[i]->rec, ACC_R});
        }
        if ((s = op_begin(ctx, acc.data(), (int)acc.size()))) return s;
        if ((s = bf_features(ctx, bf_cache(ctx), nsys, A, b, dev_feat, dev_lmax))) return s;
        return op_end(ctx, acc.data(), (int)acc.size());
    } catch (const std::bad_alloc &) {
        return set_error(APCG_ERR_OUT_OF_MEMORY, "host allocation failed");
    }
}

extern "C" apcg_status apcg_ksp_solve_batched_learned(apcg_ctx ctx, int32_t nsys, const apcg_mat *A,
                                                      const apcg_vec *b, const apcg_vec *x, double rtol,
                                                      int32_t maxit, const float *dev_params, const float *dev_mean,
                                                      const float *dev_std, const apcg_solve_opts *opts_in,
                                                      const apcg_fcg_opts *fopts_in, apcg_info info) {
    try {
        apcg_status s;
        if ((s = bf_common_checks(ctx, nsys, A, b))) return s;
        if (!x || !info || !dev_params || !dev_mean || !dev_std)
            return set_error(APCG_ERR_INVALID_ARG, "NULL argument");
        if (info->count < nsys || info->device != ctx->device)
            return set_error(APCG_ERR_INVALID_ARG, "info has fewer records than systems or another device");
        if (!(rtol >= 0.0) || !std::isfinite(rtol)) return set_error(APCG_ERR_INVALID_ARG, "rtol must be finite and >= 0");
        if (maxit < 0) return set_error(APCG_ERR_INVALID_ARG, "maxit must be >= 0");
        apcg_solve_opts opts;
        if (opts_in) opts = *opts_in;
        else apcg_solve_opts_default(&opts);
        apcg_fcg_opts fo;
        if (fopts_in) fo = *fopts_in;
        else apcg_fcg_opts_default(&fo);
        if (fo.stall_min < 1 || !(fo.stall_frac >= 0.0)) return set_error(APCG_ERR_INVALID_ARG, "bad stall window");
        if (!valid_batch_tail_rows(opts.batch_tail_tile_rows))
            return set_error(APCG_ERR_INVALID_ARG, "batch tail tile rows must be -1, 0 or a multiple of 256 in [256, 8192]");
        if (!valid_batch_tile_rows(opts.batch_tile_rows))
            return set_error(APCG_ERR_INVALID_ARG, "batch tile rows must be 0 or a multiple of 256 in [256, 8192]");
        std::vector<FSys> hs;
        std::vector<apcg_mat_s *> refill;
        int64_t ws_total = 0;
        if ((s = bf_systems(ctx, nsys, A, b, x, hs, &ws_total, refill))) return s;
        std::vector<Acc> acc;
        acc.reserve(3 * nsys + 1);
        for (int32_t i = 0; i < nsys; ++i) {
            acc.push_back({&x[i]->rec, ACC_RW});
            acc.push_back({&A[i]->rec, ACC_R});
            acc.push_back({&b[i]->rec, ACC_R});
        }
        acc.push_back({&info->rec, ACC_W});
        if ((s = op_begin(ctx, acc.data(), (int)acc.size()))) return s;
        BfCache *bc = bf_cache(ctx);
        if ((s = bf_features(ctx, bc, nsys, A, b, nullptr, nullptr))) return s;
        if ((s = mlp_infer(ctx, dev_params, dev_mean, dev_std, bc->d_X, nsys, bc->d_C))) return s;
        BfRun run;
        run.coeffs = bc->d_C;
        run.lmax = bc->d_L;
        if ((s = bf_core(ctx, bc, nsys, hs, ws_total, refill, rtol, maxit, opts, fo, run, info->d))) return s;
        return op_end(ctx, acc.data(), (int)acc.size());
    } catch (const std::bad_alloc &) {
        return set_error(APCG_ERR_OUT_OF_MEMORY, "host allocation failed");
    }
}
