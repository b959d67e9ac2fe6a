// persist.hip -- Jacobi-PCG of one small system in one persistent workgroup,
// and the latency floors it is measured against.
//
// Below about 1e5 nonzeros the paper finds the GPU iteration bound by
// latency, not bandwidth (Section 4.2): every kernel launch and every
// grid-wide reduction costs more than the data it moves.  Here a single
// 512-thread workgroup runs the whole solve in one launch: the iteration of
// the PCG loop of Section 3.3 (Jacobi preconditioning as in Section 4.1),
// its scalars and its tests never leave the workgroup.  Each thread owns R
// rows (row tid + q * 512; R <= 8, so n <= 4096), keeps their x, r, D^-1, p
// and A p entries in registers and, when the rows are short enough, their
// matrix entries as well, so after the setup an iteration reads only the
// direction vector, and x is written once, at the end:
//
//   publish p (one store per owned row into a buffer the workgroup shares),
//   barrier; w = A p for the owned rows, delta = p.w (workgroup sum, barrier);
//   alpha, x += alpha p, r -= alpha w, z = D^-1 r, z.r and the stopping norm
//   (workgroup sum, barrier); the tests; beta; p = z + beta p.
//
// Three barriers per iteration.  The two workgroup sums use separate LDS
// areas, so no barrier is needed after reading one (every reader has passed
// the next barrier before the area is written again).  The shared direction
// buffer lives in device memory that the caller provides (a workspace of n
// doubles); all of its traffic stays in the compute unit's caches.
//
// The sums run in a fixed order (a wavefront butterfly, then a butterfly over
// the 8 wavefront partials), so every thread holds the same scalars and takes
// the same decisions, and a solve is bit for bit repeatable.  The order
// differs from the multi-kernel solve's, so the two agree to rounding (both
// are checked against the oracle).
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <mutex>

#include "internal.h"

namespace apcg {
namespace {

constexpr int WT = 512;        // threads of the one workgroup (2 wavefronts per SIMD, up to 256
                               // registers per thread for the rows a thread owns)
constexpr int WNW = WT / 64;   // its wavefronts

struct WgArgs {
    const int32_t *rowptr;
    const int32_t *col;
    const double *val;
    const double *b;
    double *x;
    double *p;  // n doubles shared by the workgroup (the direction vector)
    apcg_solve_info *out;
    double rtol;
    int32_t n, maxit, x0_zero, pc, norm_pre;
};

// Workgroup sum of NV values into every thread: wavefront butterfly, one
// partial per wavefront in `area`, then the WNW partials added by a second
// butterfly in which lane l < WNW holds partial l (the other lanes 0).  An
// xor butterfly leaves every lane with the same bits (each step adds the
// same two values, only in swapped order), and every wavefront reads the same
// partials into the same lanes, so all threads hold identical sums.  The
// caller separates two uses of one area by at least one other barrier.
template <int NV>
__device__ __forceinline__ void wg_sum(double (&v)[NV], double *area) {
    const int wid = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
    for (int k = 0; k < NV; ++k) v[k] = dev::wave_sum(v[k]);
    if (lane == 0) {
#pragma unroll
        for (int k = 0; k < NV; ++k) area[k * WNW + wid] = v[k];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < NV; ++k) v[k] = dev::wave_sum(lane < WNW ? area[k * WNW + lane] : 0.0);
}

// R rows per thread; L > 0: every row has at most L entries, held in
// registers from the setup on (padding slots point at the row itself and are
// skipped); L = 0: the entries are read from the CSR arrays every iteration.
template <int R, int L>
__global__ __launch_bounds__(WT) void k_pcg_wg(WgArgs a) {
    __shared__ double red[2][4 * WNW];
    constexpr int LC = L > 0 ? L : 1;
    const int tid = threadIdx.x;
    const int n = a.n;
    double rr[R], dr[R], pr[R], wr[R], xr[R];
    int jj[R][LC];
    double aa[R][LC];
    int rs[R], rl[R];  // row start and length (rows read from the CSR arrays)

    // setup: D^-1, r0 = b - A x0, z0 = D^-1 r0, and the sums z.r, the
    // residual and reference norms, bad diagonals
    double v4[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int q = 0; q < R; ++q) {
        const int i = tid + q * WT;
        rr[q] = dr[q] = pr[q] = wr[q] = xr[q] = 0.0;
        rs[q] = rl[q] = 0;
#pragma unroll
        for (int t = 0; t < LC; ++t) {
            jj[q][t] = 0;
            aa[q][t] = 0.0;
        }
        if (i >= n) continue;
        const int s = a.rowptr[i], e = a.rowptr[i + 1];
        rs[q] = s;
        rl[q] = e - s;
        double diag = 0.0, ax = 0.0;
        bool found = false;
        if (L > 0) {
#pragma unroll
            for (int t = 0; t < LC; ++t) {
                const bool in = t < e - s;
                jj[q][t] = in ? a.col[s + t] : i;
                aa[q][t] = in ? a.val[s + t] : 0.0;
            }
#pragma unroll
            for (int t = 0; t < LC; ++t) {
                if (t < e - s) {
                    if (jj[q][t] == i) {
                        diag = aa[q][t];
                        found = true;
                    }
                    if (!a.x0_zero) ax = fma(aa[q][t], a.x[jj[q][t]], ax);
                }
            }
        } else {
            for (int k = s; k < e; ++k) {
                const int j = a.col[k];
                const double v = a.val[k];
                if (j == i) {
                    diag = v;
                    found = true;
                }
                if (!a.x0_zero) ax = fma(v, a.x[j], ax);
            }
        }
        double di = 1.0;
        if (a.pc == APCG_PC_JACOBI) {
            const bool ok = found && diag > 0.0;
            v4[3] += ok ? 0.0 : 1.0;
            di = ok ? 1.0 / diag : 0.0;
        }
        const double bi = a.b[i];
        if (!a.x0_zero) xr[q] = a.x[i];
        const double ri = a.x0_zero ? bi : bi - ax;
        rr[q] = ri;
        dr[q] = di;
        const double zi = di * ri;
        pr[q] = zi;  // p_1 = z_0 + 0 * p_0
        v4[0] = fma(zi, ri, v4[0]);
        if (a.norm_pre) {
            const double zb = di * bi;
            v4[2] = fma(zb, zb, v4[2]);
            v4[1] = fma(zi, zi, v4[1]);
        } else {
            v4[2] = fma(bi, bi, v4[2]);
            v4[1] = fma(ri, ri, v4[1]);
        }
    }
    wg_sum<4>(v4, red[0]);
    double rho = v4[0];
    double res = sqrt(v4[1]);
    const double ref = sqrt(v4[2]);
    int status = 0, its = 0;
    if (v4[3] > 0.0) status = APCG_SOLVE_SETUP_ERROR;
    else if (ref == 0.0) {
        status = APCG_SOLVE_CONVERGED;
        res = 0.0;
#pragma unroll
        for (int q = 0; q < R; ++q) xr[q] = 0.0;
    } else if (!isfinite(res) || !isfinite(ref)) status = APCG_SOLVE_NAN;
    else if (res <= a.rtol * ref) status = APCG_SOLVE_CONVERGED;
    else if (!(rho > 0.0)) status = isfinite(rho) ? APCG_SOLVE_BREAKDOWN_RZ : APCG_SOLVE_NAN;
    else if (a.maxit <= 0) status = APCG_SOLVE_MAXIT;

    for (int k = 1; !status; ++k) {
        // publish p; every thread's gathers of the previous p finished
        // before the last workgroup sum's barrier
#pragma unroll
        for (int q = 0; q < R; ++q) {
            const int i = tid + q * WT;
            if (i < n) a.p[i] = pr[q];
        }
        __syncthreads();
        double d1[1] = {0.0};
#pragma unroll
        for (int q = 0; q < R; ++q) {
            const int i = tid + q * WT;
            if (i >= n) continue;
            double sum = 0.0;
            if (L > 0) {
                double pj[LC];
#pragma unroll
                for (int t = 0; t < LC; ++t) pj[t] = a.p[jj[q][t]];
                // padding slots add 0 * p_i (a NaN or infinity there stops
                // the solve through delta anyway)
#pragma unroll
                for (int t = 0; t < LC; ++t) sum = fma(aa[q][t], pj[t], sum);
            } else {
                const int s = rs[q], len = rl[q];
                if (len <= 8) {
                    int j8[8];
                    double a8[8], p8[8];
#pragma unroll
                    for (int t = 0; t < 8; ++t) {
                        const bool in = t < len;
                        j8[t] = in ? a.col[s + t] : i;
                        a8[t] = in ? a.val[s + t] : 0.0;
                    }
#pragma unroll
                    for (int t = 0; t < 8; ++t) p8[t] = a.p[j8[t]];
#pragma unroll
                    for (int t = 0; t < 8; ++t)
                        if (t < len) sum = fma(a8[t], p8[t], sum);
                } else {
                    for (int t = s; t < s + len; ++t) sum = fma(a.val[t], a.p[a.col[t]], sum);
                }
            }
            wr[q] = sum;
            d1[0] = fma(pr[q], sum, d1[0]);
        }
        wg_sum<1>(d1, red[1]);
        const double delta = d1[0];
        if (!(delta > 0.0)) {
            status = isfinite(delta) ? APCG_SOLVE_BREAKDOWN_PAP : APCG_SOLVE_NAN;
            its = k - 1;
            break;
        }
        const double alpha = rho / delta;
        double v2[2] = {0.0, 0.0};
#pragma unroll
        for (int q = 0; q < R; ++q) {
            const int i = tid + q * WT;
            if (i >= n) continue;
            xr[q] = fma(alpha, pr[q], xr[q]);
            rr[q] = fma(-alpha, wr[q], rr[q]);
            const double zi = dr[q] * rr[q];
            v2[0] = fma(zi, rr[q], v2[0]);
            v2[1] = a.norm_pre ? fma(zi, zi, v2[1]) : fma(rr[q], rr[q], v2[1]);
        }
        wg_sum<2>(v2, red[0]);
        const double rho_new = v2[0];
        res = sqrt(v2[1]);
        its = k;
        if (!isfinite(res) || !isfinite(rho_new)) status = APCG_SOLVE_NAN;
        else if (res <= a.rtol * ref) status = APCG_SOLVE_CONVERGED;
        else if (!(rho_new > 0.0)) status = APCG_SOLVE_BREAKDOWN_RZ;
        else if (k >= a.maxit) status = APCG_SOLVE_MAXIT;
        if (!status) {
            const double beta = rho_new / rho;
            rho = rho_new;
#pragma unroll
            for (int q = 0; q < R; ++q) pr[q] = fma(beta, pr[q], dr[q] * rr[q]);
        }
    }
    // x leaves the registers once, at the end (every thread read its x0
    // entries before the first workgroup sum's barrier)
#pragma unroll
    for (int q = 0; q < R; ++q) {
        const int i = tid + q * WT;
        if (i < n) a.x[i] = xr[q];
    }
    if (tid == 0) {
        a.out->iterations = its;
        a.out->status = status;
        a.out->fcg_iterations = 0;
        a.out->half_steps = 0;
        a.out->res_norm = res;
        a.out->ref_norm = ref;
    }
}

// ------------------------------------------------------------ latency floors

__global__ void k_empty() {}

// One workgroup running `iters` iterations of the persistent solve's
// synchronisation alone: three barriers, two of them closing a workgroup sum.
__global__ __launch_bounds__(WT) void k_wg_loop(int iters, double *sink) {
    __shared__ double red[2][4 * WNW];
    double acc = 0.0;
    for (int k = 0; k < iters; ++k) {
        __syncthreads();
        double d1[1] = {1.0 + acc};
        wg_sum<1>(d1, red[1]);
        double v2[2] = {d1[0], 1.0};
        wg_sum<2>(v2, red[0]);
        acc = v2[0] * 1e-300;
    }
    if (threadIdx.x == 0) sink[0] = acc;
}

}  // namespace

// Rows per thread for n rows (0: too large for the one-workgroup solve).
int persistent_rows_per_thread(int64_t n) {
    for (int R = 1; R <= 8; R *= 2)
        if (n <= (int64_t)R * WT) return R;
    return 0;
}

// Queues the one-workgroup solve on stream st.  p: n doubles of device
// memory (the shared direction vector); maxrow: the longest row's length
// (< 0: unknown).  The caller has checked n <= APCG_PERSISTENT_MAX_N.
apcg_status launch_pcg_wg(hipStream_t st, int32_t n, const int32_t *rowptr, const int32_t *col, const double *val,
                          const double *b, double *x, double *p, double rtol, int32_t maxit, int x0_zero, int pc,
                          int norm_pre, int32_t maxrow, apcg_solve_info *out) {
    WgArgs a{rowptr, col, val, b, x, p, out, rtol, n, maxit, x0_zero, pc, norm_pre};
    const int R = persistent_rows_per_thread(n < 1 ? 1 : n);
    // matrix entries in registers when they fit without spilling (rows of
    // at most 5 entries, or of at most 7 at up to 4 rows per thread)
    const bool l5 = maxrow >= 0 && maxrow <= 5, l7 = maxrow >= 0 && maxrow <= 7;
    void (*k)(WgArgs) = nullptr;
    switch (R) {
        case 1: k = l5 ? k_pcg_wg<1, 5> : l7 ? k_pcg_wg<1, 7> : k_pcg_wg<1, 0>; break;
        case 2: k = l5 ? k_pcg_wg<2, 5> : l7 ? k_pcg_wg<2, 7> : k_pcg_wg<2, 0>; break;
        case 4: k = l5 ? k_pcg_wg<4, 5> : l7 ? k_pcg_wg<4, 7> : k_pcg_wg<4, 0>; break;
        case 8: k = l5 ? k_pcg_wg<8, 5> : k_pcg_wg<8, 0>; break;
        default: return set_error(APCG_ERR_INVALID_ARG, "system too large for the one-workgroup solve");
    }
    hipLaunchKernelGGL(k, dim3(1), dim3(WT), 0, st, a);
    APCG_CHECK_LAUNCH("k_pcg_wg");
    return APCG_SUCCESS;
}

// ------------------------------------------------- no-allocation variant
// The direction vector of apcg_ksp_solve_small_noalloc: a fixed array in the
// code object, one copy per device for the life of the process (32 KiB), so
// that the entry point allocates nothing.  Host code never passes this name
// to a kernel (on the host it is a stand-in, not a device address); it looks
// the device address up once per device and passes that.
constexpr int kNoAllocMaxN = APCG_NOALLOC_MAX_N;
static_assert(kNoAllocMaxN <= APCG_PERSISTENT_MAX_N, "the no-allocation solve is the one-workgroup solve");
static __device__ __align__(256) double scratch[kNoAllocMaxN];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double *g_scratch_ptr[kMaxDevices] = {};  // device address of `scratch`, per device

// The device address of `scratch` on `device` (looked up on the first call
// for that device, with the device current).
apcg_status scratch_address(int device, double **out) {
    if (device < 0 || device >= kMaxDevices) return set_error(APCG_ERR_INVALID_ARG, "device index out of range");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        APCG_HIP(hipSetDevice(device));
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_error(e, "hipGetSymbolAddress(scratch)");
        if (!p) return set_error(APCG_ERR_HIP, "hipGetSymbolAddress(scratch) returned NULL");
        g_scratch_ptr[device] = static_cast<double *>(p);
    }
    *out = g_scratch_ptr[device];
    return APCG_SUCCESS;
}
}  // namespace

}  // namespace apcg

using namespace apcg;

extern "C" apcg_status apcg_ksp_solve_small_noalloc(apcg_ctx ctx, int32_t n, const int32_t *rowptr,
                                                    const int32_t *col, const double *val, const double *b,
                                                    double *x, double rtol, int32_t maxit,
                                                    const apcg_solve_opts *opts, apcg_solve_info *info) {
    if (!ctx) return set_error(APCG_ERR_INVALID_ARG, "the no-allocation solve needs a context");
    if (ctx->type == APCG_STREAM_GLOBAL_BLOCKING)
        return set_error(APCG_ERR_INVALID_ARG, "the no-allocation solve needs a default-stream context");
    if (n < 0) return set_error(APCG_ERR_INVALID_ARG, "n must be >= 0");
    if (n > kNoAllocMaxN)
        return set_error(APCG_ERR_INVALID_ARG, "n exceeds APCG_NOALLOC_MAX_N (4096 rows), the no-allocation "
                                               "solve's fixed direction buffer");
    if (!rowptr || !col || !val || !b || !x || !info) return set_error(APCG_ERR_INVALID_ARG, "NULL argument");
    if (n > 0 && (uintptr_t)b < (uintptr_t)(x + n) && (uintptr_t)x < (uintptr_t)(b + n))
        return set_error(APCG_ERR_INVALID_ARG, "b and x must not share memory");
    if (maxit < 0 || !(rtol >= 0.0)) return set_error(APCG_ERR_INVALID_ARG, "maxit must be >= 0 and rtol >= 0");
    int pc = APCG_PC_JACOBI, norm_pre = 0, x0_zero = 0;
    if (opts) {
        if (opts->pc != APCG_PC_NONE && opts->pc != APCG_PC_JACOBI)
            return set_error(APCG_ERR_UNSUPPORTED, "unsupported preconditioner for the no-allocation solve");
        if (opts->norm_type != APCG_NORM_UNPRECONDITIONED && opts->norm_type != APCG_NORM_PRECONDITIONED)
            return set_error(APCG_ERR_INVALID_ARG, "unknown norm type");
        pc = opts->pc;
        norm_pre = opts->norm_type == APCG_NORM_PRECONDITIONED;
        x0_zero = opts->x0_is_zero ? 1 : 0;
    }
    double *p = nullptr;
    apcg_status s;
    if ((s = scratch_address(ctx->device, &p))) return s;
    APCG_HIP(hipSetDevice(ctx->device));
    // rows and their lengths are not known on the host: the entries are read
    // from the CSR arrays every iteration (the same sums as the register path)
    return launch_pcg_wg(ctx->stream, n, rowptr, col, val, b, x, p, rtol, maxit, x0_zero, pc, norm_pre, -1, info);
}

extern "C" apcg_status apcg_latency_floors(int32_t device, int32_t reps, double out_us[4]) {
    if (!out_us || reps < 1 || reps > 100000) return set_error(APCG_ERR_INVALID_ARG, "bad latency-floor arguments");
    apcg_status s = APCG_SUCCESS;
    int ndev = 0;
    APCG_HIP(hipGetDeviceCount(&ndev));
    if (device < 0 || device >= ndev) return set_error(APCG_ERR_INVALID_ARG, "no such device");
    APCG_HIP(hipSetDevice(device));
    hipStream_t st = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipGraph_t g = nullptr;
    hipGraphExec_t ge = nullptr;
    double *sink = nullptr;
    float ms = 0.0f;
    auto fail = [&](apcg_status code) {
        if (ge) hipGraphExecDestroy(ge);
        if (g) hipGraphDestroy(g);
        if (st) hipStreamSynchronize(st);
        if (sink) hipFree(sink);
        if (e0) hipEventDestroy(e0);
        if (e1) hipEventDestroy(e1);
        if (st) hipStreamDestroy(st);
        return code;
    };
#define FL_HIP(call)                                               \
    do {                                                           \
        hipError_t e__ = (call);                                   \
        if (e__ != hipSuccess) return fail(hip_error(e__, #call)); \
    } while (0)
    FL_HIP(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
    FL_HIP(hipEventCreate(&e0));
    FL_HIP(hipEventCreate(&e1));
    FL_HIP(hipMalloc((void **)&sink, sizeof(double)));
    // (i) back-to-back empty kernels on one stream
    hipLaunchKernelGGL(k_empty, dim3(1), dim3(64), 0, st);
    FL_HIP(hipGetLastError());
    FL_HIP(hipEventRecord(e0, st));
    for (int i = 0; i < reps; ++i) hipLaunchKernelGGL(k_empty, dim3(1), dim3(64), 0, st);
    FL_HIP(hipGetLastError());
    FL_HIP(hipEventRecord(e1, st));
    FL_HIP(hipEventSynchronize(e1));
    FL_HIP(hipEventElapsedTime(&ms, e0, e1));
    out_us[0] = 1000.0 * ms / reps;
    // (ii) a captured graph of `reps` empty kernels (at most 1000 nodes),
    // replayed: time per node
    const int nodes = reps < 1000 ? reps : 1000;
    FL_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeRelaxed));
    for (int i = 0; i < nodes; ++i) hipLaunchKernelGGL(k_empty, dim3(1), dim3(64), 0, st);
    {
        hipError_t e = hipStreamEndCapture(st, &g);
        if (e != hipSuccess) return fail(hip_error(e, "hipStreamEndCapture"));
    }
    FL_HIP(hipGraphInstantiate(&ge, g, nullptr, nullptr, 0));
    FL_HIP(hipGraphLaunch(ge, st));
    FL_HIP(hipEventRecord(e0, st));
    for (int r = 0; r < 5; ++r) FL_HIP(hipGraphLaunch(ge, st));
    FL_HIP(hipEventRecord(e1, st));
    FL_HIP(hipEventSynchronize(e1));
    FL_HIP(hipEventElapsedTime(&ms, e0, e1));
    out_us[1] = 1000.0 * ms / (5.0 * nodes);
    // (iii) one workgroup running `reps` iterations of the persistent
    // solve's synchronisation (three barriers, two workgroup sums)
    hipLaunchKernelGGL(k_wg_loop, dim3(1), dim3(WT), 0, st, 10, sink);
    FL_HIP(hipGetLastError());
    FL_HIP(hipEventRecord(e0, st));
    hipLaunchKernelGGL(k_wg_loop, dim3(1), dim3(WT), 0, st, reps, sink);
    FL_HIP(hipGetLastError());
    FL_HIP(hipEventRecord(e1, st));
    FL_HIP(hipEventSynchronize(e1));
    FL_HIP(hipEventElapsedTime(&ms, e0, e1));
    out_us[2] = 1000.0 * ms / reps;
    // (iv) host round trip: one empty kernel launched and waited for, on
    // the host's clock
    {
        const int rt = reps < 200 ? reps : 200;
        FL_HIP(hipStreamSynchronize(st));
        const auto t0 = std::chrono::steady_clock::now();
        for (int i = 0; i < rt; ++i) {
            hipLaunchKernelGGL(k_empty, dim3(1), dim3(64), 0, st);
            FL_HIP(hipGetLastError());
            FL_HIP(hipStreamSynchronize(st));
        }
        const auto t1 = std::chrono::steady_clock::now();
        out_us[3] = std::chrono::duration<double, std::micro>(t1 - t0).count() / rt;
    }
#undef FL_HIP
    s = fail(APCG_SUCCESS);
    return s;
}
