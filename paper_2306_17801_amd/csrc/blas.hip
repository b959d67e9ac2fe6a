// blas.hip -- vector kernels, device-scalar arithmetic and the plain CSR
// product behind the asynchronous Vec/Mat calls (Section 3.3: VecDotAsync,
// VecNormAsync, VecAXPYAsync, VecAYPX, VecScaleAsync, MatMult).
//
// Memory-bound kernels: each workgroup streams one contiguous chunk, and the
// XCD-aware renumbering keeps each XCD's chunks contiguous.  Scalars are read
// from device slots, never passed through the host.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "internal.h"

namespace apcg {
namespace {

constexpr int BS = 256;

using dev::Chunk;
using dev::block_chunk;

// Each thread handles UNR entries per step (UNR * BS per workgroup step),
// every load of a step issued before its first store, so several loads per
// thread are in flight: with two or fewer streams per entry, one entry per
// step leaves the HBM pipe short of requests.
constexpr int UNR = 4;

__global__ __launch_bounds__(BS) void k_dot(const double *__restrict__ x, const double *__restrict__ y, int64_t n,
                                            int64_t per_block, double *partials) {
    const Chunk c = block_chunk(n, per_block);
    double acc = 0.0;
    for (int64_t i = c.lo + threadIdx.x; i < c.hi; i += UNR * BS) {
        double xv[UNR], yv[UNR];
#pragma unroll
        for (int k = 0; k < UNR; ++k) {
            const int64_t j = i + (int64_t)k * BS;
            const bool in = j < c.hi;
            xv[k] = in ? x[j] : 0.0;
            yv[k] = in ? y[j] : 0.0;
        }
#pragma unroll
        for (int k = 0; k < UNR; ++k) acc = fma(xv[k], yv[k], acc);
    }
    double v[1] = {acc};
    dev::store_partials<BS, 1>(v, partials, gridDim.x, dev::xcd_block(blockIdx.x, gridDim.x));
}

// Second stage of the dot product: one workgroup adds the partials and
// writes the scalar (its square root for the 2-norm).
__global__ __launch_bounds__(64) void k_dot_final(const double *partials, int G, double *out, int take_sqrt) {
    double t[1];
    dev::reduce_partials<64, 1>(partials, G, t);
    if (threadIdx.x == 0) *out = take_sqrt ? sqrt(t[0]) : t[0];
}

// out[j] = f(a[j], b[j]) over the workgroup's chunk (b may alias out; a and
// b are read before out is written within each step).
template <typename F>
__device__ __forceinline__ void stream2(double *out, const double *a, const double *b, const Chunk &c, F f) {
    for (int64_t i = c.lo + threadIdx.x; i < c.hi; i += UNR * BS) {
        double av[UNR], bv[UNR];
#pragma unroll
        for (int k = 0; k < UNR; ++k) {
            const int64_t j = i + (int64_t)k * BS;
            const bool in = j < c.hi;
            av[k] = in && a ? a[j] : 0.0;
            bv[k] = in && b ? b[j] : 0.0;
        }
#pragma unroll
        for (int k = 0; k < UNR; ++k) {
            const int64_t j = i + (int64_t)k * BS;
            if (j < c.hi) out[j] = f(av[k], bv[k]);
        }
    }
}

__global__ __launch_bounds__(BS) void k_axpy(double *y, const double *a, double sign, const double *__restrict__ x,
                                             int64_t n, int64_t per_block) {
    const double s = sign * *a;
    stream2(y, x, y, block_chunk(n, per_block), [s](double xv, double yv) { return fma(s, xv, yv); });
}

__global__ __launch_bounds__(BS) void k_aypx(double *y, const double *b, const double *__restrict__ x, int64_t n,
                                             int64_t per_block) {
    const double s = *b;
    stream2(y, x, y, block_chunk(n, per_block), [s](double xv, double yv) { return fma(s, yv, xv); });
}

__global__ __launch_bounds__(BS) void k_scale(double *x, const double *a, int64_t n, int64_t per_block) {
    const double s = *a;
    stream2(x, x, nullptr, block_chunk(n, per_block), [s](double xv, double) { return s * xv; });
}

__global__ __launch_bounds__(BS) void k_copy(double *__restrict__ d, const double *__restrict__ s, int64_t n,
                                             int64_t per_block) {
    stream2(d, s, nullptr, block_chunk(n, per_block), [](double sv, double) { return sv; });
}

__global__ __launch_bounds__(BS) void k_fill(double *__restrict__ x, double v, int64_t n, int64_t per_block) {
    stream2(x, nullptr, nullptr, block_chunk(n, per_block), [v](double, double) { return v; });
}

__global__ void k_scalar_op(int op, double *out, const double *a, const double *b) {
    if (threadIdx.x != 0) return;
    const double x = *a;
    const double y = b ? *b : 0.0;
    double r = 0.0;
    switch (op) {
        case APCG_SCALAR_COPY: r = x; break;
        case APCG_SCALAR_NEG: r = -x; break;
        case APCG_SCALAR_RECIP: r = 1.0 / x; break;
        case APCG_SCALAR_SQRT: r = sqrt(x); break;
        case APCG_SCALAR_ADD: r = x + y; break;
        case APCG_SCALAR_SUB: r = x - y; break;
        case APCG_SCALAR_MUL: r = x * y; break;
        case APCG_SCALAR_DIV: r = x / y; break;
        default: r = NAN; break;
    }
    *out = r;
}

__global__ void k_scalar_set(double *out, double v) {
    if (threadIdx.x == 0) *out = v;
}

// y = A x with LPR lanes per row; rows of a workgroup form one contiguous
// range; lanes of a row add strided partial sums, then a butterfly.
template <int LPR, int TB>
__global__ __launch_bounds__(TB) void k_spmv(int32_t n, const int32_t *__restrict__ rowptr,
                                             const int32_t *__restrict__ col, const double *__restrict__ val,
                                             const double *__restrict__ x, double *__restrict__ y,
                                             int32_t rows_per_block) {
    constexpr int RPP = TB / LPR;
    const int lb = dev::xcd_block(blockIdx.x, gridDim.x);
    const int row0 = lb * rows_per_block;
    const int row1 = min(n, row0 + rows_per_block);
    const int lane = threadIdx.x % LPR, grp = threadIdx.x / LPR;
    for (int base = row0; base < row1; base += RPP) {
        const int row = base + grp;
        double sum = 0.0;
        if (row < row1) {
            const int e = rowptr[row + 1];
            for (int k = rowptr[row] + lane; k < e; k += LPR) sum = fma(val[k], x[col[k]], sum);
        }
#pragma unroll
        for (int o = LPR / 2; o > 0; o >>= 1) sum += __shfl_xor(sum, o, LPR);
        if (row < row1 && lane == 0) y[row] = sum;
    }
}

// Staged schedule (see k_pcg_product_stream): nonzeros of TB consecutive
// rows copied to LDS with coalesced loads, one row per thread.
template <int TB>
__global__ __launch_bounds__(TB) void k_spmv_stream(int32_t n, const int32_t *__restrict__ rowptr,
                                                    const int32_t *__restrict__ col, const double *__restrict__ val,
                                                    const double *__restrict__ x, double *__restrict__ y,
                                                    int32_t chunks_per_block, int32_t lds_nnz) {
    extern __shared__ double stage[];
    double *sv = stage;
    int32_t *sc = reinterpret_cast<int32_t *>(stage + lds_nnz);
    const int lb = dev::xcd_block(blockIdx.x, gridDim.x);
    const int nchunks = (n + TB - 1) / TB;
    const int c0 = lb * chunks_per_block;
    const int c1 = min(nchunks, c0 + chunks_per_block);
    for (int c = c0; c < c1; ++c) {
        const int row0 = c * TB;
        const int row1 = min(n, row0 + TB);
        const int k0 = rowptr[row0], k1 = rowptr[row1];
        __syncthreads();
        for (int k = k0 + threadIdx.x; k < k1; k += TB) {
            sv[k - k0] = __builtin_nontemporal_load(val + k);
            sc[k - k0] = __builtin_nontemporal_load(col + k);
        }
        __syncthreads();
        const int row = row0 + threadIdx.x;
        if (row < row1) {
            const int s = rowptr[row] - k0, e = rowptr[row + 1] - k0;
            double sum = 0.0;
            for (int k = s; k < e; ++k) sum = fma(sv[k], x[sc[k]], sum);
            y[row] = sum;
        }
    }
}

template <int TB>
apcg_status spmv_tb(hipStream_t s, const apcg_mat_s *A, const apcg_spmv_config &cfg, const double *x, double *y) {
    const int lpr = cfg.lanes_per_row;
    const int64_t rpp = TB / lpr;
    const int G = normalise_blocks(cfg.blocks, (A->n + rpp - 1) / rpp);
    int32_t rpb = (int32_t)((A->n + G - 1) / G);
    if (rpb < 1) rpb = 1;
#define APCG_SPMV_CASE(L)                                                                          \
    case L:                                                                                        \
        hipLaunchKernelGGL((k_spmv<L, TB>), dim3(G), dim3(TB), 0, s, A->n, A->rowptr, A->col, A->val, x, y, rpb); \
        break;
    switch (lpr) {
        APCG_SPMV_CASE(1)
        APCG_SPMV_CASE(2)
        APCG_SPMV_CASE(4)
        APCG_SPMV_CASE(8)
        APCG_SPMV_CASE(16)
        APCG_SPMV_CASE(32)
        APCG_SPMV_CASE(64)
        default: return set_error(APCG_ERR_INVALID_ARG, "unsupported lanes_per_row");
    }
#undef APCG_SPMV_CASE
    APCG_CHECK_LAUNCH("k_spmv");
    return APCG_SUCCESS;
}

}  // namespace

apcg_status launch_dot(hipStream_t s, const double *x, const double *y, int64_t n, double *out, int take_sqrt,
                       double *partials) {
    int G;
    int64_t pb;
    elementwise_grid(n, &G, &pb);
    hipLaunchKernelGGL(k_dot, dim3(G), dim3(BS), 0, s, x, y, n, pb, partials);
    APCG_CHECK_LAUNCH("k_dot");
    hipLaunchKernelGGL(k_dot_final, dim3(1), dim3(64), 0, s, (const double *)partials, G, out, take_sqrt);
    APCG_CHECK_LAUNCH("k_dot_final");
    return APCG_SUCCESS;
}

apcg_status launch_axpy(hipStream_t s, double *y, const double *a, double sign, const double *x, int64_t n) {
    if (n == 0) return APCG_SUCCESS;
    int G;
    int64_t pb;
    elementwise_grid(n, &G, &pb);
    hipLaunchKernelGGL(k_axpy, dim3(G), dim3(BS), 0, s, y, a, sign, x, n, pb);
    APCG_CHECK_LAUNCH("k_axpy");
    return APCG_SUCCESS;
}

apcg_status launch_aypx(hipStream_t s, double *y, const double *b, const double *x, int64_t n) {
    if (n == 0) return APCG_SUCCESS;
    int G;
    int64_t pb;
    elementwise_grid(n, &G, &pb);
    hipLaunchKernelGGL(k_aypx, dim3(G), dim3(BS), 0, s, y, b, x, n, pb);
    APCG_CHECK_LAUNCH("k_aypx");
    return APCG_SUCCESS;
}

apcg_status launch_scale(hipStream_t s, double *x, const double *a, int64_t n) {
    if (n == 0) return APCG_SUCCESS;
    int G;
    int64_t pb;
    elementwise_grid(n, &G, &pb);
    hipLaunchKernelGGL(k_scale, dim3(G), dim3(BS), 0, s, x, a, n, pb);
    APCG_CHECK_LAUNCH("k_scale");
    return APCG_SUCCESS;
}

apcg_status launch_copy(hipStream_t s, double *dst, const double *src, int64_t n) {
    if (n == 0) return APCG_SUCCESS;
    int G;
    int64_t pb;
    elementwise_grid(n, &G, &pb);
    hipLaunchKernelGGL(k_copy, dim3(G), dim3(BS), 0, s, dst, src, n, pb);
    APCG_CHECK_LAUNCH("k_copy");
    return APCG_SUCCESS;
}

apcg_status launch_fill(hipStream_t s, double *x, double v, int64_t n) {
    if (n == 0) return APCG_SUCCESS;
    int G;
    int64_t pb;
    elementwise_grid(n, &G, &pb);
    hipLaunchKernelGGL(k_fill, dim3(G), dim3(BS), 0, s, x, v, n, pb);
    APCG_CHECK_LAUNCH("k_fill");
    return APCG_SUCCESS;
}

apcg_status launch_scalar_op(hipStream_t s, int op, double *out, const double *a, const double *b) {
    hipLaunchKernelGGL(k_scalar_op, dim3(1), dim3(64), 0, s, op, out, a, b);
    APCG_CHECK_LAUNCH("k_scalar_op");
    return APCG_SUCCESS;
}

apcg_status launch_scalar_set(hipStream_t s, double *out, double v) {
    hipLaunchKernelGGL(k_scalar_set, dim3(1), dim3(64), 0, s, out, v);
    APCG_CHECK_LAUNCH("k_scalar_set");
    return APCG_SUCCESS;
}

// y = A x with configuration cfg (the matrix's own, or the CSR one chosen
// for a lone product on a sliced schedule).
static apcg_status spmv_with(hipStream_t s, const apcg_mat_s *A, const apcg_spmv_config &cfg, const double *x,
                             double *y) {
    if (cfg.schedule == APCG_SPMV_STREAM && stream_fits(A, cfg.block_size)) {
        const int tb = cfg.block_size;
        const int64_t nchunks = ((int64_t)A->n + tb - 1) / tb;
        const int G = normalise_blocks(cfg.blocks, nchunks);
        const int32_t cpb = (int32_t)std::max<int64_t>(1, (nchunks + G - 1) / G);
        const int32_t lds_nnz = (int32_t)std::max<int64_t>(2, ((A->max_block_nnz[tb == 512 ? 1 : 0] + 1) / 2) * 2);
        const size_t lds = (size_t)lds_nnz * (sizeof(double) + sizeof(int32_t));
        if (tb == 512)
            hipLaunchKernelGGL((k_spmv_stream<512>), dim3(G), dim3(512), lds, s, A->n, A->rowptr, A->col, A->val, x,
                               y, cpb, lds_nnz);
        else
            hipLaunchKernelGGL((k_spmv_stream<256>), dim3(G), dim3(256), lds, s, A->n, A->rowptr, A->col, A->val, x,
                               y, cpb, lds_nnz);
        APCG_CHECK_LAUNCH("k_spmv_stream");
        return APCG_SUCCESS;
    }
    if (cfg.block_size == 512) return spmv_tb<512>(s, A, cfg, x, y);
    return spmv_tb<256>(s, A, cfg, x, y);
}

apcg_status launch_spmv(hipStream_t s, const apcg_mat_s *A, const double *x, double *y) {
    if (A->n == 0) return APCG_SUCCESS;
    if (A->cfg.schedule == APCG_SPMV_SELL || A->cfg.schedule == APCG_SPMV_SDIA || A->cfg.schedule == APCG_SPMV_DIA) {
        // The sliced copies are refilled per solve, not per product: a lone
        // product reads the CSR arrays with row groups of the configured
        // block size and grid, lanes per row from the mean row length.
        const double mean = (double)A->nnz / (double)A->n;
        const int lpr = mean <= 8 ? 1 : mean <= 16 ? 2 : mean <= 32 ? 4 : mean <= 64 ? 8 : 16;
        const apcg_spmv_config cfg{lpr, A->cfg.block_size, A->cfg.blocks, APCG_SPMV_ROWGROUP};
        return spmv_with(s, A, cfg, x, y);
    }
    return spmv_with(s, A, A->cfg, x, y);
}

}  // namespace apcg
