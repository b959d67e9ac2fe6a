// pcg.hip -- the preconditioned conjugate-gradient hot path with every
// scalar on the device (the PCG loop of Section 3.3 with Jacobi
// preconditioning as in Section 4.1).
//
// One iteration k is two kernels:
//
//   product P_k: every workgroup first reduces the update partials of
//       iteration k-1 (rho_{k-1} = z.r, ||r||^2) and applies the tests of
//       iteration k-1 (NaN, convergence, r.z breakdown, iteration limit); if
//       none fires, beta_k = rho_{k-1} / rho_{k-2}, and the workgroup computes
//       p_k = D^-1 r + beta_k p_{k-1} while gathering it, w = A p_k and its
//       share of delta_k = p_k . w.
//   update U_k:  every workgroup reduces the delta partials of P_k, stops on
//       delta <= 0, else alpha_k = rho_{k-1} / delta_k; x += alpha p,
//       r -= alpha w, z = D^-1 r (stored, so the next product gathers z and
//       p_{k-1}) and its shares of z.r, ||r||^2.
//
// There is no atomic and no fence in any kernel: a reduction's first stage
// writes one partial per workgroup, and the consuming kernel (which starts
// after the producer has finished) re-adds them in a fixed order in every
// workgroup, so all workgroups reach bit-identical scalars and identical
// decisions.  On CDNA each agent-scope release of a workgroup writes back its
// XCD's L2, which made a last-workgroup-finishes reduction cost several times
// the kernel's own streaming time; the kernel boundary does that once.
//
// Scalars live in a device SolveState.  A kernel never writes a field its own
// workgroups read: product P_k reads record rec[(k-1)&1] and writes rec[k&1];
// the stop flag is monotonic (0 -> 1) and every workgroup that could observe
// either value takes the same decision.  Once the flag is set every later
// kernel returns at once, so work queued after convergence is a no-op and x is
// exactly the converged iterate (the device-side convergence check the paper
// leaves for future work in Section 5).  p is double-buffered: iteration k
// reads p[(k+1)&1] and writes p[k&1], so a K-iteration graph with K even can
// be replayed.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <map>
#include <cmath>
#include <cstring>

#include "internal.h"

namespace apcg {

struct PcgRecord {  // written by P_k into rec[k & 1]
    double rho;     // rho_{k-1} = z_{k-1} . r_{k-1}
    double beta;    // beta_k
    double res;     // stopping norm after iteration k-1
    int32_t k;
    int32_t pad;
};

struct SolveState {
    PcgRecord rec[2];
    double ref, rtol;     // reference norm, relative tolerance (set by init)
    int32_t maxit, zero_x;
    double out_res;       // terminal results
    int32_t out_its, out_status;
    int32_t flag;         // 1 once a terminal state is reached
    int32_t hist_cap;     // > 0: record alpha_k / beta_k (Lanczos data)
    double *hist;         // [0, cap): alpha_k; [cap, 2 cap): beta_k
};
static_assert(sizeof(SolveState) <= 256, "solve state exceeds its allocation");

namespace {

constexpr int VB = 256;  // block size of the vector-shaped kernels
// partials layout inside the context's buffer (slices of kMaxBlocks doubles)
constexpr int kSliceResidual = 0;  // 4 slices: z.r, ||.||^2, reference^2, bad rows
constexpr int kSliceDelta = 4;     // 1 slice: p.Ap

// The direction entry p_j = z_j + beta p_old_j.  z = D^-1 r is stored (as
// the rounded products d_j r_j) by the setup and update kernels, so the
// product kernels gather two arrays (z, p_old) instead of three, and the
// stored p and every gathered p agree bit for bit.
__device__ __forceinline__ double pdir(double z, double beta, double pold) { return fma(beta, pold, z); }

// Tests applied after iteration m (oracle order: NaN, convergence, r.z
// breakdown, iteration limit).  Returns the status bit or 0.
__device__ __forceinline__ int iteration_status(double rho, double res, const SolveState *st, int m) {
    if (!isfinite(res) || !isfinite(rho)) return APCG_SOLVE_NAN;
    if (res <= st->rtol * st->ref) return APCG_SOLVE_CONVERGED;
    if (!(rho > 0.0)) return APCG_SOLVE_BREAKDOWN_RZ;
    if (m >= st->maxit) return APCG_SOLVE_MAXIT;
    return 0;
}

__device__ __forceinline__ void terminate(SolveState *st, int its, int status, double res) {
    st->out_its = its;
    st->out_status = status;
    st->out_res = res;
    st->flag = 1;
}

// ----------------------------------------------------------------- setup
// dinv = 1/diag(A) (or 1), r0 = b - A x0 (or b), z0 = dinv r0, p_old = 0; partials of
// z0.r0, residual norm^2, reference norm^2 and the count of bad diagonals.
__global__ __launch_bounds__(VB) void k_pcg_init(int32_t n, const int32_t *__restrict__ rowptr,
                                                 const int32_t *__restrict__ col, const double *__restrict__ val,
                                                 const double *__restrict__ b, double *__restrict__ x,
                                                 double *__restrict__ r, double *__restrict__ dinv,
                                                 double *__restrict__ z, double *__restrict__ pold,
                                                 double *partials, int64_t per_block, int x0_zero, int pc,
                                                 int norm_pre, const int32_t *gate) {
    if (gate && !gate[0]) return;  // gated off: the solve is a no-op
    const dev::Chunk c = dev::block_chunk(n, per_block);
    double rz = 0.0, nres = 0.0, nref = 0.0, bad = 0.0;
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
        if (x0_zero) x[i] = 0.0;  // x is not read when x0 is taken as zero
        const double zi = di * ri;
        z[i] = zi;
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
    double v[4] = {rz, nres, nref, bad};
    dev::store_partials<VB, 4>(v, partials, gridDim.x, dev::xcd_block(blockIdx.x, gridDim.x));
}

// One workgroup: reference norm, initial tests, record 0.
__global__ __launch_bounds__(64) void k_pcg_init_final(SolveState *st, const double *partials, int G, double rtol,
                                                       int32_t maxit, double *hist, int32_t hist_cap,
                                                       const int32_t *gate) {
    if (gate && !gate[0]) {  // gated off: stop before the first iteration, nothing computed
        if (threadIdx.x == 0) {
            st->zero_x = 0;
            st->hist = nullptr;
            st->hist_cap = 0;
            terminate(st, 0, 0, 0.0);
        }
        return;
    }
    if (gate) maxit = gate[1];
    double v[4];
    dev::reduce_partials<64, 4>(partials, G, v);
    if (threadIdx.x != 0) return;
    const double rho = v[0], res = sqrt(v[1]), ref = sqrt(v[2]);
    st->ref = ref;
    st->rtol = rtol;
    st->maxit = maxit;
    st->zero_x = 0;
    st->flag = 0;
    st->out_its = 0;
    st->out_status = 0;
    st->out_res = res;
    st->rec[0] = PcgRecord{rho, 0.0, res, 0, 0};
    st->rec[1] = PcgRecord{0.0, 0.0, 0.0, -1, 0};
    st->hist = hist;
    st->hist_cap = hist ? hist_cap : 0;
    int status = 0;
    if (v[3] > 0.0) status = APCG_SOLVE_SETUP_ERROR;
    else if (ref == 0.0) {
        status = APCG_SOLVE_CONVERGED;  // b = 0: the solution is x = 0
        st->zero_x = 1;
    } else if (!isfinite(res) || !isfinite(ref)) status = APCG_SOLVE_NAN;
    else if (res <= rtol * ref) status = APCG_SOLVE_CONVERGED;
    else if (!(rho > 0.0)) status = isfinite(rho) ? APCG_SOLVE_BREAKDOWN_RZ : APCG_SOLVE_NAN;
    else if (maxit <= 0) status = APCG_SOLVE_MAXIT;
    if (status) terminate(st, 0, status, st->zero_x ? 0.0 : res);
}

// x0 was given and b turned out to be zero: x = 0.
__global__ __launch_bounds__(VB) void k_pcg_zero_x_if(double *__restrict__ x, int64_t n, int64_t per_block,
                                                      const SolveState *st) {
    if (!st->zero_x) return;
    const dev::Chunk c = dev::block_chunk(n, per_block);
    for (int64_t i = c.lo + threadIdx.x; i < c.hi; i += VB) x[i] = 0.0;
}

// ----------------------------------------------------------------- product
// Scalar step at the start of product P_k, identical in every workgroup:
// tests of iteration k-1 and beta_k.  Returns false when the solve has
// stopped (the caller returns).  tune != 0: autotuner timing only (the
// reduction runs, its result is unused, beta = 0.5, no state is written).
template <int TB>
__device__ __forceinline__ bool product_prologue(SolveState *st, const double *part_res, int g_res, int parity,
                                                 int tune, double *beta_out) {
    if (tune) {
        double v[2];
        dev::reduce_partials<TB, 2>(part_res, g_res, v);
        *beta_out = v[0] == 12345.678 ? 0.25 : 0.5;  // keeps the timed reduction alive
        return true;
    }
    if (st->flag) return false;
    const PcgRecord prev = st->rec[parity ^ 1];
    const int k = prev.k + 1;
    double rho = prev.rho, res = prev.res, beta = 0.0;
    if (k > 1) {
        double v[2];
        dev::reduce_partials<TB, 2>(part_res, g_res, v);
        rho = v[0];
        res = sqrt(v[1]);
        const int status = iteration_status(rho, res, st, k - 1);
        if (status) {
            if (blockIdx.x == 0 && threadIdx.x == 0) terminate(st, k - 1, status, res);
            return false;
        }
        beta = rho / prev.rho;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        st->rec[parity] = PcgRecord{rho, beta, res, k, 0};
        if (k > 1 && k - 1 <= st->hist_cap) st->hist[st->hist_cap + k - 2] = beta;  // beta after iteration k-1
    }
    *beta_out = beta;
    return true;
}

// parity = k & 1.  tune != 0 (autotuner only): no tests, beta = 0.5, no state
// written, the kernel always runs.
template <int LPR, int TB>
__global__ __launch_bounds__(TB) void k_pcg_product(int32_t n, const int32_t *__restrict__ rowptr,
                                                    const int32_t *__restrict__ col, const double *__restrict__ val,
                                                    const double *__restrict__ z,
                                                    const double *__restrict__ pold, double *__restrict__ pnew,
                                                    double *__restrict__ w, SolveState *st, const double *part_res,
                                                    int g_res, double *part_delta, int32_t rows_per_block,
                                                    int parity, int tune, int32_t /*lds_nnz: staged only*/) {
    double beta;
    if (!product_prologue<TB>(st, part_res, g_res, parity, tune, &beta)) return;
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
                sum = fma(val[k], pdir(z[j], beta, pold[j]), sum);
            }
        }
#pragma unroll
        for (int o = LPR / 2; o > 0; o >>= 1) sum += __shfl_xor(sum, o, LPR);
        if (row < row1 && lane == 0) {
            const double pi = pdir(z[row], beta, pold[row]);
            pnew[row] = pi;
            w[row] = sum;
            acc = fma(pi, sum, acc);
        }
    }
    double v[1] = {acc};
    dev::store_partials<TB, 1>(v, part_delta, gridDim.x, lb);
}


// Row sum of A p for one row whose nonzeros are staged in LDS at [s, e).
// Rows of at most 8 entries issue all gathers before the first multiply-add
// (the padded slots gather the row's own entry and are not added); longer
// rows take the plain loop.  Both paths add in column-storage order, so the
// result does not depend on which one ran.
__device__ __forceinline__ double staged_row_product(const double *sv, const int32_t *sc, int s, int e, int row,
                                                     const double *__restrict__ z, const double *__restrict__ pold,
                                                     double beta) {
    const int len = e - s;
    double sum = 0.0;
    if (len <= 8) {
        int jj[8];
        double aa[8], pj[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const bool in = q < len;
            jj[q] = in ? sc[s + q] : row;
            aa[q] = in ? sv[s + q] : 0.0;
        }
#pragma unroll
        for (int q = 0; q < 8; ++q) pj[q] = pdir(z[jj[q]], beta, pold[jj[q]]);
#pragma unroll
        for (int q = 0; q < 8; ++q)
            if (q < len) sum = fma(aa[q], pj[q], sum);
    } else {
        for (int k = s; k < e; ++k) {
            const int j = sc[k];
            sum = fma(sv[k], pdir(z[j], beta, pold[j]), sum);
        }
    }
    return sum;
}

// Staged schedule: each workgroup walks its contiguous run of TB-row chunks;
// per chunk the nonzeros are moved to LDS with coalesced (non-temporal)
// loads, then thread t reduces row t of the chunk.  With one row per thread,
// neighbouring lanes gather neighbouring entries of z and p_old, which
// coalesces for banded/stencil matrices.  The chunk loop is software
// pipelined: the next chunk's nonzeros are loaded into registers (PF per
// thread) while the current chunk is reduced, so staging does not serialise
// with the gathers.  lds_nnz (>= the largest chunk) sizes the LDS stage and
// PF * TB >= lds_nnz.
template <int TB, int PF>
__global__ __launch_bounds__(TB) void k_pcg_product_stream(int32_t n, const int32_t *__restrict__ rowptr,
                                                           const int32_t *__restrict__ col,
                                                           const double *__restrict__ val,
                                                           const double *__restrict__ z,
                                                           const double *__restrict__ pold, double *__restrict__ pnew,
                                                           double *__restrict__ w, SolveState *st,
                                                           const double *part_res, int g_res, double *part_delta,
                                                           int32_t chunks_per_block, int parity, int tune,
                                                           int32_t lds_nnz) {
    double beta;
    if (!product_prologue<TB>(st, part_res, g_res, parity, tune, &beta)) return;
    extern __shared__ double stage[];
    double *sv = stage;
    int32_t *sc = reinterpret_cast<int32_t *>(stage + lds_nnz);
    const int lb = dev::xcd_block(blockIdx.x, gridDim.x);
    const int nchunks = (n + TB - 1) / TB;
    const int c0 = lb * chunks_per_block;
    const int c1 = min(nchunks, c0 + chunks_per_block);
    double pv[PF];
    int32_t pc[PF];
    int pk0 = 0, pcount = 0;
    auto prefetch = [&](int c) {
        const int row0 = c * TB;
        const int row1 = min(n, row0 + TB);
        pk0 = rowptr[row0];
        pcount = rowptr[row1] - pk0;
#pragma unroll
        for (int q = 0; q < PF; ++q) {
            const int k = q * TB + threadIdx.x;
            if (k < pcount) {
                pv[q] = __builtin_nontemporal_load(val + pk0 + k);
                pc[q] = __builtin_nontemporal_load(col + pk0 + k);
            }
        }
    };
    if (c0 < c1) prefetch(c0);
    double acc = 0.0;
    for (int c = c0; c < c1; ++c) {
        const int row0 = c * TB;
        const int row1 = min(n, row0 + TB);
        const int k0 = pk0;
        __syncthreads();  // the previous chunk's LDS reads are done
#pragma unroll
        for (int q = 0; q < PF; ++q) {
            const int k = q * TB + threadIdx.x;
            if (k < pcount) {
                sv[k] = pv[q];
                sc[k] = pc[q];
            }
        }
        __syncthreads();
        if (c + 1 < c1) prefetch(c + 1);  // in flight during the gathers below
        const int row = row0 + threadIdx.x;
        if (row < row1) {
            const double sum =
                staged_row_product(sv, sc, rowptr[row] - k0, rowptr[row + 1] - k0, row, z, pold, beta);
            const double pi = pdir(z[row], beta, pold[row]);
            pnew[row] = pi;
            w[row] = sum;
            acc = fma(pi, sum, acc);
        }
    }
    double v[1] = {acc};
    dev::store_partials<TB, 1>(v, part_delta, gridDim.x, lb);
}

// Sliced schedule (SELL-64): wavefront v of a workgroup takes slices
// s0 + v, s0 + v + TB/64, ... of the workgroup's contiguous range, lane l
// reduces row 64 s + l.  meta[2 s] is the slice's offset and meta[2 s + 1]
// its width W; entry k of lane l sits at offset + 64 k + l, so each load of
// a column index or value is one coalesced 512-byte access.  Padding entries
// have column -1 and are not added: each row adds its own entries in
// column-storage order, as in the other schedules.
// NARROW (every slice at most 8 wide): software pipelined -- the next
// slice's column and value loads are issued before the current slice's
// gathers, so the HBM stream of the matrix overlaps the cache-bound gathers.
// Otherwise slices are reduced one entry at a time.
template <int TB, int NARROW>
__global__ __launch_bounds__(TB) void k_pcg_product_sell(int32_t n, const int32_t *__restrict__ meta,
                                                         const int32_t *__restrict__ scol,
                                                         const double *__restrict__ sval, const double *__restrict__ z,
                                                         const double *__restrict__ pold, double *__restrict__ pnew,
                                                         double *__restrict__ w, SolveState *st,
                                                         const double *part_res, int g_res, double *part_delta,
                                                         int32_t slices_per_block, int parity, int tune,
                                                         int32_t /*lds_nnz: staged only*/) {
    const int lb = dev::xcd_block(blockIdx.x, gridDim.x);
    const int nsl = (n + 63) / 64;
    const int s0 = lb * slices_per_block;
    const int s1 = min(nsl, s0 + slices_per_block);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    constexpr int STEP = TB / 64;
    int jn[8];
    double an[8];
    auto load = [&](int sl) {
        const int off = meta[2 * sl], W = meta[2 * sl + 1];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const bool in = k < W;
            jn[k] = in ? __builtin_nontemporal_load(scol + off + 64 * k + lane) : -1;
            an[k] = in ? __builtin_nontemporal_load(sval + off + 64 * k + lane) : 0.0;
        }
    };
    // the first slice's matrix loads do not depend on beta: issued before the
    // prologue's reduction so that its latency overlaps them
    if (NARROW && s0 + wave < s1) load(s0 + wave);
    double beta;
    if (!product_prologue<TB>(st, part_res, g_res, parity, tune, &beta)) return;
    double acc = 0.0;
    if (NARROW) {
        for (int sl = s0 + wave; sl < s1; sl += STEP) {
            int jj[8];
            double aa[8], pj[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                jj[k] = jn[k];
                aa[k] = an[k];
            }
            if (sl + STEP < s1) load(sl + STEP);  // in flight during the gathers below
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                const int j = jj[k] >= 0 ? jj[k] : 0;  // padding gathers row 0 and is not added
                pj[k] = pdir(z[j], beta, pold[j]);
            }
            double sum = 0.0;
#pragma unroll
            for (int k = 0; k < 8; ++k)
                if (jj[k] >= 0) sum = fma(aa[k], pj[k], sum);
            const int row = sl * 64 + lane;
            if (row < n) {
                const double pi = pdir(z[row], beta, pold[row]);
                pnew[row] = pi;
                w[row] = sum;
                acc = fma(pi, sum, acc);
            }
        }
    } else {
        for (int sl = s0 + wave; sl < s1; sl += STEP) {
            const int off = meta[2 * sl], W = meta[2 * sl + 1];
            double sum = 0.0;
            for (int k = 0; k < W; ++k) {
                const int j = __builtin_nontemporal_load(scol + off + 64 * k + lane);
                if (j >= 0)
                    sum = fma(__builtin_nontemporal_load(sval + off + 64 * k + lane), pdir(z[j], beta, pold[j]), sum);
            }
            const int row = sl * 64 + lane;
            if (row < n) {
                const double pi = pdir(z[row], beta, pold[row]);
                pnew[row] = pi;
                w[row] = sum;
                acc = fma(pi, sum, acc);
            }
        }
    }
    double v[1] = {acc};
    dev::store_partials<TB, 1>(v, part_delta, gridDim.x, lb);
}

// Fills the sliced copy from the CSR arrays: thread (slice, lane) copies its
// row's entries to offset + 64 k + lane and pads to the slice's width with
// column -1 and value 0.
__global__ __launch_bounds__(256) void k_sell_fill(int32_t n, const int32_t *__restrict__ rowptr,
                                                   const int32_t *__restrict__ col, const double *__restrict__ val,
                                                   const int32_t *__restrict__ meta, int32_t *__restrict__ scol,
                                                   double *__restrict__ sval) {
    const int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t nsl = ((int64_t)n + 63) / 64;
    if (g >= nsl * 64) return;
    const int sl = (int)(g >> 6), lane = (int)(g & 63);
    const int row = sl * 64 + lane;
    const int off = meta[2 * sl], W = meta[2 * sl + 1];
    int s = 0, len = 0;
    if (row < n) {
        s = rowptr[row];
        len = rowptr[row + 1] - s;
    }
    for (int k = 0; k < W; ++k) {
        const bool in = k < len;
        scol[off + 64 * k + lane] = in ? col[s + k] : -1;
        sval[off + 64 * k + lane] = in ? val[s + k] : 0.0;
    }
}

// Sliced-diagonal schedule (SDIA): wavefront v of a workgroup takes slices
// s0 + v, s0 + v + TB/64, ... of the workgroup's contiguous range, lane l
// reduces row 64 s + l.  Slice s has W offset slots s*W .. s*W+W-1 (sorted
// column offsets, a 64-bit row mask each, mask 0 beyond the slice's own
// offsets; W in {8, 16, 32}) and value slots s*U .. s*U+U-1 of 64 values,
// one per lane.  The row adds the entries its mask bits select in offset
// order, i.e. in column order, with one fused multiply-add each: the same sum
// as the row-per-thread and sliced schedules.  Branch-free: every load is
// issued unconditionally (value slot clamped to U-1, the gather index of an
// absent entry pointed at the row itself) and absent entries are dropped by
// selects, so all W slots' loads of a slice are in flight together; the
// offsets and masks of 8 slots are one scalar load each.
// W == 8: software pipelined -- the next slice's offsets, masks and values
// are loaded before the current slice's gathers.
template <int TB, int W>
__global__ __launch_bounds__(TB) void k_pcg_product_sdia(int32_t n, const int32_t *__restrict__ soff,
                                                         const int32_t *__restrict__ smask_words,
                                                         const double *__restrict__ sval, const double *__restrict__ z,
                                                         const double *__restrict__ pold, double *__restrict__ pnew,
                                                         double *__restrict__ w, SolveState *st,
                                                         const double *part_res, int g_res, double *part_delta,
                                                         int32_t slices_per_block, int parity, int tune,
                                                         int32_t U) {
    const uint64_t *smask = reinterpret_cast<const uint64_t *>(smask_words);
    const int lb = dev::xcd_block(blockIdx.x, gridDim.x);
    const int nsl = (n + 63) / 64;
    const int s0 = lb * slices_per_block;
    const int s1 = min(nsl, s0 + slices_per_block);
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    constexpr int STEP = TB / 64;
    int on[W];
    uint64_t mn[W];
    double an[W];
    auto load = [&](int sl) {
        const int32_t *o = soff + (int64_t)sl * W;
        const uint64_t *m = smask + (int64_t)sl * W;
        const double *v = sval + (int64_t)sl * U * 64 + lane;
#pragma unroll
        for (int k = 0; k < W; ++k) {
            on[k] = o[k];
            mn[k] = m[k];
            an[k] = __builtin_nontemporal_load(v + (int64_t)min(k, U - 1) * 64);
        }
    };
    // the first slice's loads do not depend on beta: issued before the
    // prologue's reduction so that its latency overlaps them
    if (W == 8 && s0 + wave < s1) load(s0 + wave);
    double beta;
    if (!product_prologue<TB>(st, part_res, g_res, parity, tune, &beta)) return;
    double acc = 0.0;
    for (int sl = s0 + wave; sl < s1; sl += STEP) {
        const int row = sl * 64 + lane;
        const int rc = min(row, n - 1);
        int oc[W];
        uint64_t mc[W];
        double ac[W];
        __builtin_amdgcn_s_setprio(2);  // the slice's loads issued ahead of other waves' arithmetic
        if (W == 8) {
#pragma unroll
            for (int k = 0; k < W; ++k) {
                oc[k] = on[k];
                mc[k] = mn[k];
                ac[k] = an[k];
            }
            if (sl + STEP < s1) load(sl + STEP);  // in flight during the gathers below
        } else {
            load(sl);
#pragma unroll
            for (int k = 0; k < W; ++k) {
                oc[k] = on[k];
                mc[k] = mn[k];
                ac[k] = an[k];
            }
        }
        double zj[W], pj[W];
        bool in[W];
#pragma unroll
        for (int k = 0; k < W; ++k) {
            in[k] = (mc[k] >> lane) & 1ull;
            const int j = in[k] ? row + oc[k] : rc;
            zj[k] = z[j];
            pj[k] = pold[j];
        }
        const double zi = z[rc], po = pold[rc];
        __builtin_amdgcn_s_setprio(0);
        double sum = 0.0;
#pragma unroll
        for (int k = 0; k < W; ++k) {
            const double t = fma(ac[k], pdir(zj[k], beta, pj[k]), sum);
            sum = in[k] ? t : sum;
        }
        // stored for the rows past n of the last slice too (workspace
        // vectors padded to whole slices): no branch for the next slice to
        // wait behind
        const double pi = pdir(zi, beta, po);
        pnew[row] = pi;
        w[row] = sum;
        acc = row < n ? fma(pi, sum, acc) : acc;
    }
    double v[1] = {acc};
    dev::store_partials<TB, 1>(v, part_delta, gridDim.x, lb);
}

// Sliced diagonals, plane marching (lanes_per_row = seg > 1 selects it when
// the pattern has a plane stride): the slices form Ps columns (Ps = the
// pattern's plane stride in slices, i.e. the offset +-64 Ps is a
// neighbouring plane); task (segment g, column c) walks slices
// s_j = j Ps + c for j in [g seg, (g+1) seg).  The window of offset +64 Ps
// of slice s_j is slice s_{j+1}'s own window: loaded once, it serves as the
// +plane neighbour now and as the own window (and then the -plane
// neighbour) of the next slices, so those windows are neither gathered
// through the cache twice nor dependent on the slice's offset loads.  Other
// offsets are gathered as in k_pcg_product_sdia; the sums are bitwise the
// same.  shape = U | seg << 8 | Ps << 16.  Tasks are spread over the grid
// (task += waves in the grid).
// Symmetric values (the flag behind the partner table: set by the analysis
// for a structurally symmetric pattern, cleared by the check kernel when a
// refill finds the values unequal): an entry left of the diagonal, (i, i - q), is read as its
// transpose (i - q, i) from that row's slot of offset +q: one load at the
// partner slot's address, of a line the product reads anyway -- for q = 64
// Ps the previous slice's +plane slot, which this wavefront loaded one step
// earlier; for the other offsets the same slice or a slice a few rows back
// -- so only the slots on and right of the diagonal stream from memory.  The
// values are bitwise the same, and so is the sum.
// The marching tasks of one wavefront; returns its share of p.Ap.  SYM:
// entries left of the diagonal read as their transposes (one load each, at
// the partner slot's address; no branches on the offsets).
template <int TB, int W, int UC, bool SYM>
__device__ __forceinline__ double march_tasks(int32_t n, const int32_t *__restrict__ soff,
                                              const uint64_t *__restrict__ smask, const double *__restrict__ sval,
                                              const double *__restrict__ z, const double *__restrict__ pold,
                                              double *__restrict__ pnew, double *__restrict__ w, int lb, double beta,
                                              int U, int seg, int Ps) {
    const int nsl = (n + 63) / 64;
    const int nz = (nsl + Ps - 1) / Ps;  // planes (the last may be partial)
    const int nseg = (nz + seg - 1) / seg;
    const int ntask = Ps * nseg;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int nwaves = gridDim.x * (TB / 64);
    const int up = 64 * Ps;
    const int32_t *part = soff + (int64_t)nsl * W;
    double acc = 0.0;
    for (int task = lb * (TB / 64) + wave; task < ntask; task += nwaves) {
        const int c = task % Ps, g = task / Ps;
        const int j0 = g * seg, j1 = min(nz, j0 + seg);
        // own and -plane windows of the first slice
        int row = (j0 * Ps + c) * 64 + lane;
        int rc = min(row, n - 1);
        double zo = z[rc], po = pold[rc];
        const int rp = max(rc - up, 0);
        double zm = z[rp], pm = pold[rp];
        for (int j = j0; j < j1; ++j) {
            const int sl = j * Ps + c;
            if (sl >= nsl) break;  // the partial last plane
            row = sl * 64 + lane;
            rc = min(row, n - 1);
            const int32_t *o = soff + (int64_t)sl * W;
            const uint64_t *m = smask + (int64_t)sl * W;
            const int32_t *pt = part + (int64_t)sl * W;
            __builtin_amdgcn_s_setprio(2);  // the slice's loads issued ahead of other waves' arithmetic
            const int rn = min(rc + up, n - 1);
            const double zn = z[rn], pn = pold[rn];  // +plane window = the next slice's own
            int oc[W], qc[W];
            uint64_t mc[W];
            double ac[W];
            bool in[W];
#pragma unroll
            for (int k = 0; k < UC; ++k) {
                oc[k] = o[k];
                mc[k] = m[k];
                qc[k] = SYM ? pt[k] : 0;
            }
#pragma unroll
            for (int k = 0; k < UC; ++k) {
                in[k] = (mc[k] >> lane) & 1ull;
                if constexpr (SYM) {
                    // own slot, or for an entry left of the diagonal the
                    // slot of its transpose (row row + offset); bit
                    // arithmetic rather than selects keeps this one
                    // straight-line block whose loads are all in flight
                    const int lowm = oc[k] >> 31;  // all ones left of the diagonal
                    const int r = sl * 64 + lane + (in[k] ? (oc[k] & lowm) : 0);
                    const int ps = (lane >= ((-oc[k]) & 63) ? qc[k] : (qc[k] >> 8)) & 0xff;
                    const int slot = (ps & lowm) | (min(k, U - 1) & ~lowm);
                    ac[k] = sval[((int64_t)(r >> 6) * U + slot) * 64 + (r & 63)];
                } else {
                    ac[k] = __builtin_nontemporal_load(sval + ((int64_t)sl * U + min(k, U - 1)) * 64 + lane);
                }
            }
            double zj[W], pj[W];
#pragma unroll
            for (int k = 0; k < UC; ++k) {
                const bool carried = oc[k] == up || oc[k] == -up || oc[k] == 0;
                const int jx = (in[k] && !carried) ? row + oc[k] : rc;
                const double zg = carried ? 0.0 : z[jx], pg = carried ? 0.0 : pold[jx];
                zj[k] = oc[k] == up ? zn : oc[k] == -up ? zm : oc[k] == 0 ? zo : zg;
                pj[k] = oc[k] == up ? pn : oc[k] == -up ? pm : oc[k] == 0 ? po : pg;
            }
            __builtin_amdgcn_s_setprio(0);
            double sum = 0.0;
#pragma unroll
            for (int k = 0; k < UC; ++k) {
                const double t = fma(ac[k], pdir(zj[k], beta, pj[k]), sum);
                sum = in[k] ? t : sum;
            }
            // stored for the rows past n of the last slice too: p and w
            // are workspace vectors padded to whole slices, so the stores
            // need no branch (whose join would make the next slice wait for
            // them)
            const double pi = pdir(zo, beta, po);
            pnew[row] = pi;
            w[row] = sum;
            acc = row < n ? fma(pi, sum, acc) : acc;
            zm = zo;
            pm = po;
            zo = zn;
            po = pn;
        }
    }
    return acc;
}

// UC: offset slots walked per slice, a compile-time bound >= U (the slots
// past U hold no entry in any slice): 5 or 7 for the 2D and 3D 5/7-point
// patterns keeps the unused slot's loads and registers out of the kernel,
// and at most 72 VGPRs (asked for below) let 7 wavefronts share a SIMD.
template <int TB, int W, int UC>
__global__ __launch_bounds__(TB) __attribute__((amdgpu_waves_per_eu(UC <= 7 ? 7 : 1))) void k_pcg_product_sdia_march(int32_t n, const int32_t *__restrict__ soff,
                                                               const int32_t *__restrict__ smask_words,
                                                               const double *__restrict__ sval,
                                                               const double *__restrict__ z,
                                                               const double *__restrict__ pold,
                                                               double *__restrict__ pnew, double *__restrict__ w,
                                                               SolveState *st, const double *part_res, int g_res,
                                                               double *part_delta, int32_t /*unused*/, int parity,
                                                               int tune, int32_t shape) {
    const uint64_t *smask = reinterpret_cast<const uint64_t *>(smask_words);
    const int U = shape & 0xff, seg = (shape >> 8) & 0xff, Ps = (shape >> 16) & 0xffff;
    const int lb = dev::xcd_block(blockIdx.x, gridDim.x);
    const int nsl = (n + 63) / 64;
    const int sym = __builtin_amdgcn_readfirstlane(soff[2 * (int64_t)nsl * W]);
    double beta;
    if (!product_prologue<TB>(st, part_res, g_res, parity, tune, &beta)) return;
    const double acc = sym ? march_tasks<TB, W, UC, true>(n, soff, smask, sval, z, pold, pnew, w, lb, beta, U, seg, Ps)
                           : march_tasks<TB, W, UC, false>(n, soff, smask, sval, z, pold, pnew, w, lb, beta, U, seg, Ps);
    double v[1] = {acc};
    dev::store_partials<TB, 1>(v, part_delta, gridDim.x, lb);
}

// Fills the sliced-diagonal value copy from the CSR values: thread
// (slice, lane) walks its row's entries in order, one per set mask bit, and
// writes 0 to the slots its row does not hold.
__global__ __launch_bounds__(256) void k_sdia_fill(int32_t n, const int32_t *__restrict__ rowptr,
                                                   const double *__restrict__ val, const uint64_t *__restrict__ smask,
                                                   int32_t U, int32_t MP, double *__restrict__ sval) {
    const int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t nsl = ((int64_t)n + 63) / 64;
    if (g >= nsl * 64) return;
    const int64_t sl = g >> 6;
    const int lane = (int)(g & 63);
    const int64_t row = sl * 64 + lane;
    int64_t e = row < n ? rowptr[row] : 0;
    for (int k = 0; k < U; ++k) {
        const bool in = (smask[sl * MP + k] >> lane) & 1ull;
        sval[(sl * U + k) * 64 + lane] = in ? val[e] : 0.0;
        e += in ? 1 : 0;
    }
}

// Value symmetry of a structurally symmetric pattern: thread (slice, lane)
// compares each of its row's entries left of the diagonal, bit for bit, with
// its transpose's copy (the partner slot, see sdia_analyse) and clears the
// flag on any difference, so that the products read every slot themselves.
// The flag is only ever cleared on the device (the analysis sets it once):
// a product running on another stream never sees it set for values found
// unequal, and after such a refill the matrix keeps reading every slot.
__global__ __launch_bounds__(256) void k_sdia_symcheck(int32_t n, const int32_t *__restrict__ soff,
                                                       const uint64_t *__restrict__ smask, int32_t U, int32_t MP,
                                                       const double *__restrict__ sval, int32_t *__restrict__ symflag) {
    const int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t nsl = ((int64_t)n + 63) / 64;
    if (g >= nsl * 64) return;
    const int64_t sl = g >> 6;
    const int lane = (int)(g & 63);
    const int32_t *part = soff + nsl * MP;
    bool same = true;
    for (int k = 0; k < U; ++k) {
        const int32_t o = soff[sl * MP + k];
        if (o >= 0 || !((smask[sl * MP + k] >> lane) & 1ull)) continue;
        const int64_t r = sl * 64 + lane + o;  // the transpose's row, >= 0 for a present entry
        const int pk = part[sl * MP + k];
        const int slot = lane >= ((-o) & 63) ? (pk & 0xff) : ((pk >> 8) & 0xff);
        const double a = sval[(sl * U + k) * 64 + lane];
        const double t = sval[((r >> 6) * U + slot) * 64 + (r & 63)];
        same = same && __double_as_longlong(a) == __double_as_longlong(t);
    }
    if (!same) symflag[0] = 0;
}

// ------------------------------------------------------------- diagonals
// The matrix as at most 9 diagonals (the distinct offsets o_k = column - row,
// ascending): val[k][i] = a_{i, i + o_k}, 0 where row i has no such entry.
// Table tab: offsets [0..8], for a negative offset the diagonal holding its
// transpose's values [9..17] (-1: none), the value-symmetry flag [18].

// Row i of A p for rows lo + tid, lo + tid + TB, ... < hi (the rows of the
// row-per-thread schedule at lanes_per_row 1, in the same order), with
// p_j = z_j + beta pold_j formed while gathering.  Every address is the row
// plus a constant: the diagonal values at row i, the vectors at i + o_k
// (clamped into [0, n); an absent entry's value is 0, so the clamped gather
// only multiplies into an exact zero).  SYM: the value at a negative offset
// -q is diagonal +q's value at row i - q (0 above the first row).  The sum
// runs over the diagonals in offset order with one FMA each; the absent
// entries add exact zeros (a sum started at +0 is never -0), so it is bitwise
// the CSR row sum.  Returns the thread's share of p.Ap.
template <int TB, int ND, bool SYM>
__device__ __forceinline__ double dia_rows(int32_t n, const int (&off)[ND], const int (&prt)[ND], int nd,
                                           const double *__restrict__ dval, int64_t stride,
                                           const double *__restrict__ z, const double *__restrict__ pold,
                                           double *__restrict__ pnew, double *__restrict__ w, double beta, int lo,
                                           int hi) {
    double acc = 0.0;
    for (int row = lo + (int)threadIdx.x; row < hi; row += TB) {
        double a[ND], g[ND];
#pragma unroll
        for (int k = 0; k < ND; ++k) {
            if (k < nd) {
                const int o = off[k];
                const int j = min(max(row + o, 0), n - 1);
                g[k] = pdir(z[j], beta, pold[j]);
                if (SYM && o < 0) {
                    const int src = row + o;
                    const double t = dval[(int64_t)prt[k] * stride + max(src, 0)];
                    a[k] = src >= 0 ? t : 0.0;
                } else {
                    a[k] = dval[(int64_t)k * stride + row];
                }
            } else {
                a[k] = 0.0;
                g[k] = 0.0;
            }
        }
        double sum = 0.0;
#pragma unroll
        for (int k = 0; k < ND; ++k) sum = fma(a[k], g[k], sum);
        const double pi = pdir(z[row], beta, pold[row]);
        pnew[row] = pi;
        w[row] = sum;
        acc = fma(pi, sum, acc);
    }
    return acc;
}

// Product with the diagonal layout: a1 unused, a2 = the diagonals,
// lds_nnz = the diagonal count the kernel walks (ND).  rows_per_block is a
// multiple of 64, so every wavefront's loads are contiguous windows.
template <int TB, int ND>
__global__ __launch_bounds__(TB) void k_pcg_product_dia(int32_t n, const int32_t *__restrict__ tab,
                                                        const int32_t * /*unused*/, const double *__restrict__ dval,
                                                        const double *__restrict__ z,
                                                        const double *__restrict__ pold, double *__restrict__ pnew,
                                                        double *__restrict__ w, SolveState *st,
                                                        const double *part_res, int g_res, double *part_delta,
                                                        int32_t rows_per_block, int parity, int tune,
                                                        int32_t nd_walked) {
    double beta;
    if (!product_prologue<TB>(st, part_res, g_res, parity, tune, &beta)) return;
    const int64_t stride = ((int64_t)n + 63) / 64 * 64;
    int off[ND], prt[ND];
#pragma unroll
    for (int k = 0; k < ND; ++k) {
        off[k] = __builtin_amdgcn_readfirstlane(tab[k]);
        prt[k] = __builtin_amdgcn_readfirstlane(tab[9 + k]);
    }
    const int nd = __builtin_amdgcn_readfirstlane(tab[19]);
    const int sym = __builtin_amdgcn_readfirstlane(tab[18]);
    const int lb = dev::xcd_block(blockIdx.x, gridDim.x);
    const int lo = lb * rows_per_block, hi = min(n, lo + rows_per_block);
    const double acc = sym ? dia_rows<TB, ND, true>(n, off, prt, nd, dval, stride, z, pold, pnew, w, beta, lo, hi)
                           : dia_rows<TB, ND, false>(n, off, prt, nd, dval, stride, z, pold, pnew, w, beta, lo, hi);
    double v[1] = {acc};
    dev::store_partials<TB, 1>(v, part_delta, gridDim.x, lb);
}

// Diagonals with plane marching (lanes_per_row = seg > 1 selects it when the
// offsets hold a pair +-64 Ps, the plane stride in 64-row slices): the
// slices form Ps columns and a task (wavefront) walks seg consecutive
// slices of one column, one plane apart, as the sliced-diagonal marching
// product does.  The window of offset +64 Ps (z and p_old of the next
// slice's rows) is loaded once and serves as the +plane neighbour now, then
// as the next slice's own window and then as its -plane neighbour; with
// symmetric values the -plane entry is the previous slice's +plane value,
// kept in a register.  Every other address is the row plus a constant the
// whole wavefront shares, so no load waits for per-slice offsets: the
// values of the diagonals on and right of the main one (of all of them
// without symmetry) and the gathers of the remaining offsets are issued
// together.  The sum runs over the diagonals in offset order with one FMA
// each, as in k_pcg_product_dia, so the two kernels give the same bits.
// shape = ND walked | seg << 8 | Ps << 16.
template <int TB, int ND, bool SYM>
__device__ __forceinline__ double dia_march_tasks(int32_t n, const int (&off)[ND], const int (&prt)[ND], int nd,
                                                  const double *__restrict__ dval, int64_t stride,
                                                  const double *__restrict__ z, const double *__restrict__ pold,
                                                  double *__restrict__ pnew, double *__restrict__ w, int lb,
                                                  double beta, int seg, int Ps) {
    const int nsl = (n + 63) / 64;
    const int nz = (nsl + Ps - 1) / Ps;  // planes (the last may be partial)
    const int nseg = (nz + seg - 1) / seg;
    const int ntask = Ps * nseg;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int nwaves = gridDim.x * (TB / 64);
    const int up = 64 * Ps;
    int kup = -1;  // the +plane diagonal (its value carries to the next slice's -plane entry)
#pragma unroll
    for (int k = 0; k < ND; ++k)
        if (k < nd && off[k] == up) kup = k;
    double acc = 0.0;
    for (int task = lb * (TB / 64) + wave; task < ntask; task += nwaves) {
        const int c = task % Ps, g = task / Ps;
        const int j0 = g * seg, j1 = min(nz, j0 + seg);
        int row = (j0 * Ps + c) * 64 + lane;
        int rc = min(row, n - 1);
        double zo = z[rc], po = pold[rc];  // own window
        const int rp = max(rc - up, 0);
        double zm = z[rp], pm = pold[rp];  // -plane window
        double aprev = 0.0;  // the +plane value of row - up
        if (SYM && kup >= 0 && row - up >= 0) aprev = dval[(int64_t)kup * stride + (row - up)];
        for (int j = j0; j < j1; ++j) {
            const int sl = j * Ps + c;
            if (sl >= nsl) break;  // the partial last plane
            row = sl * 64 + lane;
            rc = min(row, n - 1);
            __builtin_amdgcn_s_setprio(2);  // the slice's loads issued ahead of other waves' arithmetic
            const int rn = min(rc + up, n - 1);
            const double zn = z[rn], pn = pold[rn];  // +plane window = the next slice's own
            double a[ND], zg[ND], pg[ND];
#pragma unroll
            for (int k = 0; k < ND; ++k) {
                const int o = off[k];
                const bool live = k < nd;
                const bool carried = o == up || o == -up || o == 0;
                if (SYM && o < 0) {
                    // the transpose's value, diagonal +q at row - q (the
                    // -plane one carried from the previous slice)
                    const int src = row + o;
                    const double t = (o == -up || !live) ? 0.0 : dval[(int64_t)prt[k] * stride + max(src, 0)];
                    a[k] = !live ? 0.0 : o == -up ? aprev : (src >= 0 ? t : 0.0);
                } else {
                    a[k] = live ? dval[(int64_t)k * stride + row] : 0.0;
                }
                const int jx = (live && !carried) ? min(max(row + o, 0), n - 1) : rc;
                const double zl = z[jx], pl = pold[jx];
                zg[k] = !live ? 0.0 : o == up ? zn : o == -up ? zm : o == 0 ? zo : zl;
                pg[k] = !live ? 0.0 : o == up ? pn : o == -up ? pm : o == 0 ? po : pl;
            }
            __builtin_amdgcn_s_setprio(0);
            double sum = 0.0;
#pragma unroll
            for (int k = 0; k < ND; ++k) sum = fma(a[k], pdir(zg[k], beta, pg[k]), sum);
            // workspace vectors are padded to whole slices: the rows past n
            // of the last slice store padding, without a branch
            const double pi = pdir(zo, beta, po);
            pnew[row] = pi;
            w[row] = sum;
            acc = row < n ? fma(pi, sum, acc) : acc;
            if (SYM && kup >= 0) {
#pragma unroll
                for (int k = 0; k < ND; ++k)
                    if (k == kup) aprev = a[k];
            }
            zm = zo;
            pm = po;
            zo = zn;
            po = pn;
        }
    }
    return acc;
}

template <int TB, int ND>
__global__ __launch_bounds__(TB) void k_pcg_product_dia_march(int32_t n, const int32_t *__restrict__ tab,
                                                              const int32_t * /*unused*/,
                                                              const double *__restrict__ dval,
                                                              const double *__restrict__ z,
                                                              const double *__restrict__ pold,
                                                              double *__restrict__ pnew, double *__restrict__ w,
                                                              SolveState *st, const double *part_res, int g_res,
                                                              double *part_delta, int32_t /*unused*/, int parity,
                                                              int tune, int32_t shape) {
    const int seg = (shape >> 8) & 0xff, Ps = (shape >> 16) & 0xffff;
    double beta;
    if (!product_prologue<TB>(st, part_res, g_res, parity, tune, &beta)) return;
    const int64_t stride = ((int64_t)n + 63) / 64 * 64;
    int off[ND], prt[ND];
#pragma unroll
    for (int k = 0; k < ND; ++k) {
        off[k] = __builtin_amdgcn_readfirstlane(tab[k]);
        prt[k] = __builtin_amdgcn_readfirstlane(tab[9 + k]);
    }
    const int nd = __builtin_amdgcn_readfirstlane(tab[19]);
    const int sym = __builtin_amdgcn_readfirstlane(tab[18]);
    const int lb = dev::xcd_block(blockIdx.x, gridDim.x);
    const double acc =
        sym ? dia_march_tasks<TB, ND, true>(n, off, prt, nd, dval, stride, z, pold, pnew, w, lb, beta, seg, Ps)
            : dia_march_tasks<TB, ND, false>(n, off, prt, nd, dval, stride, z, pold, pnew, w, lb, beta, seg, Ps);
    double v[1] = {acc};
    dev::store_partials<TB, 1>(v, part_delta, gridDim.x, lb);
}

// Refills the diagonals from the CSR values: thread i walks row i's entries
// (columns strictly increasing, every offset one of the table's) against the
// ascending offsets and writes every diagonal's value of row i (0 for rows
// >= n and for the diagonals past nd).
__global__ __launch_bounds__(256) void k_dia_fill(int32_t n, const int32_t *__restrict__ rowptr,
                                                  const int32_t *__restrict__ col, const double *__restrict__ val,
                                                  const int32_t *__restrict__ tab, int32_t ndt,
                                                  double *__restrict__ dval) {
    const int64_t stride = ((int64_t)n + 63) / 64 * 64;
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= stride) return;
    const int nd = tab[19];
    int e = i < n ? rowptr[i] : 0;
    const int end = i < n ? rowptr[i + 1] : 0;
    for (int k = 0; k < ndt; ++k) {
        double v = 0.0;
        if (k < nd && e < end && (int64_t)col[e] == i + tab[k]) {
            v = val[e];
            ++e;
        }
        dval[k * stride + i] = v;
    }
}

// Clears the value-symmetry flag when an entry left of the diagonal differs
// in any bit from its transpose's (diagonal +q at row i - q); queued after
// every refill of a matrix with a symmetric offset set.  The flag is never
// set on the device, so a product on another context's stream never sees it
// set for values found unequal.
__global__ __launch_bounds__(256) void k_dia_symcheck(int32_t n, int32_t *__restrict__ tab,
                                                      const double *__restrict__ dval) {
    const int64_t stride = ((int64_t)n + 63) / 64 * 64;
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const int nd = tab[19];
    bool same = true;
    for (int k = 0; k < nd; ++k) {
        const int o = tab[k];
        if (o >= 0) continue;
        const int64_t src = i + o;
        const double a = dval[k * stride + i];
        const double t = src >= 0 ? dval[(int64_t)tab[9 + k] * stride + src] : 0.0;
        same = same && __double_as_longlong(a) == __double_as_longlong(t);
    }
    if (!same) tab[18] = 0;
}

// ----------------------------------------------------------------- update
__global__ __launch_bounds__(VB) void k_pcg_update(int64_t n, double *__restrict__ x, double *__restrict__ r,
                                                   const double *__restrict__ p, const double *__restrict__ w,
                                                   const double *__restrict__ dinv, double *__restrict__ z,
                                                   SolveState *st,
                                                   const double *part_delta, int g_delta, double *part_res,
                                                   int64_t per_block, int parity, int norm_pre, int tune) {
    // a thread's entries i0, i0 + VB, i0 + 2 VB, ... in groups of UN whose
    // loads are all issued before the group's arithmetic (same order of
    // accumulation as one entry at a time); the first group's loads do not
    // depend on alpha and are issued before the reduction of p.Ap so that
    // its latency overlaps them
    constexpr int UN = 4;
    const dev::Chunk c = dev::block_chunk(n, per_block);
    const int64_t i0 = c.lo + threadIdx.x;
    double xs[UN], rs[UN], ps[UN], ws[UN], ds[UN];
    auto load = [&](int64_t ib) {
#pragma unroll
        for (int u = 0; u < UN; ++u) {
            const int64_t i = ib + (int64_t)u * VB;
            const bool ok = i < c.hi;
            xs[u] = ok ? x[i] : 0.0;
            rs[u] = ok ? r[i] : 0.0;
            ps[u] = ok ? p[i] : 0.0;
            ws[u] = ok ? w[i] : 0.0;
            ds[u] = ok ? dinv[i] : 0.0;
        }
    };
    load(i0);
    double alpha = 0.0;
    double d[1];
    if (tune) {
        dev::reduce_partials<VB, 1>(part_delta, g_delta, d);  // timed like the real kernel
        if (d[0] == 12345.678) alpha = 1e-300;
    } else {
        if (st->flag) return;
        const PcgRecord rec = st->rec[parity];
        dev::reduce_partials<VB, 1>(part_delta, g_delta, d);
        const double delta = d[0];
        if (!(delta > 0.0)) {
            if (blockIdx.x == 0 && threadIdx.x == 0)
                terminate(st, rec.k - 1, isfinite(delta) ? APCG_SOLVE_BREAKDOWN_PAP : APCG_SOLVE_NAN, rec.res);
            return;
        }
        alpha = rec.rho / delta;
        if (blockIdx.x == 0 && threadIdx.x == 0 && rec.k <= st->hist_cap) st->hist[rec.k - 1] = alpha;
    }
    double rz = 0.0, nn = 0.0;
    for (int64_t ib = i0; ib < c.hi; ib += (int64_t)UN * VB) {
        if (ib != i0) load(ib);
#pragma unroll
        for (int u = 0; u < UN; ++u) {
            const int64_t i = ib + (int64_t)u * VB;
            if (i < c.hi) {
                const double xi = fma(alpha, ps[u], xs[u]);
                const double ri = fma(-alpha, ws[u], rs[u]);
                x[i] = xi;
                r[i] = ri;
                const double zi = ds[u] * ri;
                z[i] = zi;
                rz = fma(zi, ri, rz);
                nn = norm_pre ? fma(zi, zi, nn) : fma(ri, ri, nn);
            }
        }
    }
    double v[2] = {rz, nn};
    dev::store_partials<VB, 2>(v, part_res, gridDim.x, dev::xcd_block(blockIdx.x, gridDim.x));
}

// Applies the tests of the last launched iteration when no later product
// kernel did, then copies the terminal state into the caller's info record.
__global__ __launch_bounds__(64) void k_pcg_finish(SolveState *st, const double *part_res, int g_res,
                                                   apcg_solve_info *out) {
    if (!st->flag) {
        const int q = st->rec[1].k > st->rec[0].k ? 1 : 0;
        const PcgRecord last = st->rec[q];
        double v[2];
        dev::reduce_partials<64, 2>(part_res, g_res, v);
        if (threadIdx.x == 0) {
            const double res = sqrt(v[1]);
            int status = iteration_status(v[0], res, st, last.k);
            if (!status) status = APCG_SOLVE_MAXIT;  // the host stopped at maxit
            terminate(st, last.k, status, res);
        }
    }
    if (threadIdx.x != 0) return;
    out->iterations = st->out_its;
    out->status = st->out_status;
    out->fcg_iterations = 0;
    out->half_steps = 0;
    out->res_norm = st->out_res;
    out->ref_norm = st->ref;
}

__global__ __launch_bounds__(VB) void k_tune_fill(double *r, double *dinv, double *p, double *z, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * VB + threadIdx.x; i < n; i += (int64_t)gridDim.x * VB) {
        r[i] = 1.0 + 1e-3 * (double)(i % 97);
        dinv[i] = 0.25;
        p[i] = 0.125;
        z[i] = 0.25 * r[i];
    }
}

using ProductFn = void (*)(int32_t, const int32_t *, const int32_t *, const double *, const double *,
                           const double *, double *, double *, SolveState *, const double *, int, double *, int32_t,
                           int, int, int32_t);

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

// Staged kernels by the prefetch depth PF (nonzeros per thread): the
// smallest PF with PF * TB >= lds_nnz keeps the register count low.
template <int TB>
ProductFn stream_fn(int32_t lds_nnz) {
    const int need = (lds_nnz + TB - 1) / TB;
    if (need <= 4) return k_pcg_product_stream<TB, 4>;
    if (need <= 8) return k_pcg_product_stream<TB, 8>;
    if (need <= 12) return k_pcg_product_stream<TB, 12>;
    if (TB == 512 || need <= 16) return k_pcg_product_stream<TB, (TB == 512 ? 11 : 16)>;
    return k_pcg_product_stream<TB, 21>;  // 21 * 256 >= kStreamMaxNnz
}

ProductFn product_fn(const apcg_spmv_config &cfg, int32_t lds_nnz, int32_t sell_maxw, int32_t sdia_mp,
                     int32_t sdia_ps) {
    if (cfg.schedule == APCG_SPMV_DIA) {
        const bool b512 = cfg.block_size == 512;
        if (cfg.lanes_per_row > 1 && (lds_nnz >> 16) > 0) {  // plane marching
            const int nd = lds_nnz & 0xff;
            if (nd <= 5) return b512 ? k_pcg_product_dia_march<512, 5> : k_pcg_product_dia_march<256, 5>;
            if (nd <= 7) return b512 ? k_pcg_product_dia_march<512, 7> : k_pcg_product_dia_march<256, 7>;
            return b512 ? k_pcg_product_dia_march<512, 9> : k_pcg_product_dia_march<256, 9>;
        }
        if (lds_nnz <= 5) return b512 ? k_pcg_product_dia<512, 5> : k_pcg_product_dia<256, 5>;
        if (lds_nnz <= 7) return b512 ? k_pcg_product_dia<512, 7> : k_pcg_product_dia<256, 7>;
        return b512 ? k_pcg_product_dia<512, 9> : k_pcg_product_dia<256, 9>;
    }
    if (cfg.schedule == APCG_SPMV_SDIA) {
        const bool b512 = cfg.block_size == 512;
        if (cfg.lanes_per_row > 1 && sdia_ps > 0) {  // plane marching
            const int U = lds_nnz & 0xff;
            if (sdia_mp == 8 && U <= 5)
                return b512 ? k_pcg_product_sdia_march<512, 8, 5> : k_pcg_product_sdia_march<256, 8, 5>;
            if (sdia_mp == 8 && U <= 7)
                return b512 ? k_pcg_product_sdia_march<512, 8, 7> : k_pcg_product_sdia_march<256, 8, 7>;
            if (sdia_mp == 8) return b512 ? k_pcg_product_sdia_march<512, 8, 8> : k_pcg_product_sdia_march<256, 8, 8>;
            if (sdia_mp == 16)
                return b512 ? k_pcg_product_sdia_march<512, 16, 16> : k_pcg_product_sdia_march<256, 16, 16>;
            return b512 ? k_pcg_product_sdia_march<512, 32, 32> : k_pcg_product_sdia_march<256, 32, 32>;
        }
        if (sdia_mp == 8) return b512 ? k_pcg_product_sdia<512, 8> : k_pcg_product_sdia<256, 8>;
        if (sdia_mp == 16) return b512 ? k_pcg_product_sdia<512, 16> : k_pcg_product_sdia<256, 16>;
        return b512 ? k_pcg_product_sdia<512, 32> : k_pcg_product_sdia<256, 32>;
    }
    if (cfg.schedule == APCG_SPMV_SELL) {
        if (sell_maxw <= 8)
            return cfg.block_size == 512 ? k_pcg_product_sell<512, 1> : k_pcg_product_sell<256, 1>;
        return cfg.block_size == 512 ? k_pcg_product_sell<512, 0> : k_pcg_product_sell<256, 0>;
    }
    if (cfg.schedule == APCG_SPMV_STREAM) {
        if (cfg.block_size == 512) return stream_fn<512>(lds_nnz);
        return stream_fn<256>(lds_nnz);
    }
    return cfg.block_size == 512 ? product_fn_tb<512>(cfg.lanes_per_row) : product_fn_tb<256>(cfg.lanes_per_row);
}

// Launch geometry of one solve.
struct Plan {
    int32_t n;
    ProductFn prod;
    const int32_t *a0, *a1;  // matrix arrays the product reads: CSR rowptr, col -- or slice meta, column copy
    const double *a2;        //   CSR values -- or the value copy
    int tb;
    int g_prod;
    int32_t rpb;  // rows (row groups), chunks (staged) or slices (sliced) per workgroup
    int g_vec;
    int64_t pb_vec;
    int32_t lds_nnz;     // staged schedule: LDS entries per workgroup; sliced diagonals: value slots per slice
    size_t lds_bytes;
};

// Vector-shaped kernels: at most 1024 workgroups of VB threads, chunks a
// multiple of 64 entries; few workgroups keep the partials every consumer
// workgroup re-adds short.
void vector_grid(int64_t n, int *G, int64_t *per_block) {
    const int64_t units = (n + 63) / 64;
    *G = normalise_blocks(1024, units);
    int64_t pb = (n + *G - 1) / *G;
    *per_block = std::max<int64_t>(64, ((pb + 63) / 64) * 64);
}

apcg_status make_plan(const apcg_mat_s *A, const apcg_spmv_config &cfg, Plan *pl) {
    pl->n = A->n;
    pl->tb = cfg.block_size == 512 ? 512 : 256;
    if (cfg.schedule == APCG_SPMV_STREAM && !stream_fits(A, pl->tb))
        return set_error(APCG_ERR_UNSUPPORTED, "rows too long for the staged schedule");
    pl->lds_nnz = 0;
    pl->lds_bytes = 0;
    pl->a0 = A->rowptr;
    pl->a1 = A->col;
    pl->a2 = A->val;
    if (cfg.schedule == APCG_SPMV_DIA) {
        if (A->dia_state != 1 || !A->dia_val)
            return set_error(APCG_ERR_INVALID_STATE, "diagonal copy not prepared");
        pl->a0 = A->dia_tab;
        pl->a1 = nullptr;
        pl->a2 = A->dia_val;
        const int64_t units = ((int64_t)A->n + 63) / 64;  // 64-row chunks
        if (cfg.lanes_per_row > 1 && A->dia_ps > 0) {  // plane marching: seg planes per task
            const int64_t seg = cfg.lanes_per_row, ps = A->dia_ps, waves = pl->tb / 64;
            const int64_t nz = (units + ps - 1) / ps, tasks = ps * ((nz + seg - 1) / seg);
            pl->g_prod = normalise_blocks(kMaxBlocks, (tasks + waves - 1) / waves);
            pl->rpb = 0;
            pl->lds_nnz = A->dia_ndt | (int32_t)(seg << 8) | (int32_t)(ps << 16);
        } else {
            pl->g_prod = normalise_blocks(cfg.blocks, (units * 64 + pl->tb - 1) / pl->tb);
            const int64_t upb = (units + pl->g_prod - 1) / pl->g_prod;
            pl->rpb = (int32_t)std::max<int64_t>(64, upb * 64);
            pl->lds_nnz = A->dia_ndt;
        }
    } else if (cfg.schedule == APCG_SPMV_SDIA) {
        if (A->sdia_state != 1 || !A->sdia_val)
            return set_error(APCG_ERR_INVALID_STATE, "sliced-diagonal copy not prepared");
        pl->a0 = A->sdia_off;
        pl->a1 = reinterpret_cast<const int32_t *>(A->sdia_msk);
        pl->a2 = A->sdia_val;
        const int64_t nsl = ((int64_t)A->n + 63) / 64;
        const int64_t waves = pl->tb / 64;
        if (cfg.lanes_per_row > 1 && A->sdia_ps > 0) {  // plane marching: seg planes per task
            const int64_t seg = cfg.lanes_per_row, ps = A->sdia_ps;
            const int64_t nz = (nsl + ps - 1) / ps, tasks = ps * ((nz + seg - 1) / seg);
            pl->g_prod = normalise_blocks(kMaxBlocks, (tasks + waves - 1) / waves);
            pl->rpb = 0;
            pl->lds_nnz = A->sdia_u | (int32_t)(seg << 8) | (int32_t)(ps << 16);
        } else {
            pl->g_prod = normalise_blocks(cfg.blocks, (nsl + waves - 1) / waves);
            pl->rpb = (int32_t)std::max<int64_t>(1, (nsl + pl->g_prod - 1) / pl->g_prod);
            pl->lds_nnz = A->sdia_u;  // the kernel's value slots per slice
        }
    } else if (cfg.schedule == APCG_SPMV_SELL) {
        if (!A->sell_meta) return set_error(APCG_ERR_INVALID_STATE, "sliced copy not prepared");
        pl->a0 = A->sell_meta;
        pl->a1 = A->sell_col;
        pl->a2 = A->sell_val;
        const int64_t nsl = ((int64_t)A->n + 63) / 64;
        const int64_t waves = pl->tb / 64;
        pl->g_prod = normalise_blocks(cfg.blocks, (nsl + waves - 1) / waves);
        pl->rpb = (int32_t)std::max<int64_t>(1, (nsl + pl->g_prod - 1) / pl->g_prod);
    } else if (cfg.schedule == APCG_SPMV_STREAM) {
        const int64_t most = A->max_block_nnz[pl->tb == 512 ? 1 : 0];
        pl->lds_nnz = (int32_t)std::max<int64_t>(2, ((most + 1) / 2) * 2);  // keeps the int32 stage 8-byte aligned
        pl->lds_bytes = (size_t)pl->lds_nnz * (sizeof(double) + sizeof(int32_t));
        const int64_t nchunks = ((int64_t)A->n + pl->tb - 1) / pl->tb;
        pl->g_prod = normalise_blocks(cfg.blocks, nchunks);
        pl->rpb = (int32_t)std::max<int64_t>(1, (nchunks + pl->g_prod - 1) / pl->g_prod);
    } else {
        const int64_t rpp = pl->tb / cfg.lanes_per_row;
        pl->g_prod = normalise_blocks(cfg.blocks, (A->n + rpp - 1) / rpp);
        int64_t rpb = ((int64_t)A->n + pl->g_prod - 1) / pl->g_prod;
        pl->rpb = (int32_t)std::max<int64_t>(1, rpb);
    }
    pl->prod = product_fn(cfg, pl->lds_nnz, A->sell_maxw, A->sdia_mp, A->sdia_ps);
    if (!pl->prod) return set_error(APCG_ERR_INVALID_ARG, "unsupported lanes_per_row");
    vector_grid(A->n, &pl->g_vec, &pl->pb_vec);
    return APCG_SUCCESS;
}

// Allocates the matrix's sliced copy on first use (uploading the slice
// table once) and queues its refill from the CSR arrays on stream s.
apcg_status prepare_sell(apcg_mat_s *A, hipStream_t s) {
    if (A->sell_entries < 0) return set_error(APCG_ERR_UNSUPPORTED, "matrix too large for the sliced layout");
    const int64_t nsl = ((int64_t)A->n + 63) / 64;
    if (!A->sell_meta) {
        const int64_t ent = std::max<int64_t>(A->sell_entries, 1);
        APCG_HIP(hipMalloc((void **)&A->sell_meta, sizeof(int32_t) * std::max<int64_t>(2 * nsl, 2)));
        APCG_HIP(hipMalloc((void **)&A->sell_col, sizeof(int32_t) * ent));
        APCG_HIP(hipMalloc((void **)&A->sell_val, sizeof(double) * ent));
        if (nsl > 0) {
            g_counters.h2d_copies++;
            APCG_HIP(hipMemcpyAsync(A->sell_meta, A->sell_meta_h.data(), sizeof(int32_t) * 2 * nsl,
                                    hipMemcpyHostToDevice, s));
            g_counters.host_syncs++;
            APCG_HIP(hipStreamSynchronize(s));  // once per matrix
        }
    }
    if (nsl > 0) {
        const int64_t blocks = (nsl * 64 + 255) / 256;
        hipLaunchKernelGGL(k_sell_fill, dim3((unsigned)blocks), dim3(256), 0, s, A->n, A->rowptr, A->col, A->val,
                           (const int32_t *)A->sell_meta, A->sell_col, A->sell_val);
        APCG_CHECK_LAUNCH("k_sell_fill");
    }
    return APCG_SUCCESS;
}

}  // namespace

// Builds the sliced-diagonal offsets and masks on the host from a copy of
// the CSR pattern (once per matrix) and allocates the device copies.  Leaves
// sdia_state -1 with a reason when the layout does not apply.
apcg_status sdia_analyse(apcg_mat_s *A) {
    if (A->sdia_state != 0) return APCG_SUCCESS;
    auto reject = [&](const char *why) {
        A->sdia_state = -1;
        A->sdia_reason = why;
        return APCG_SUCCESS;
    };
    const int64_t n = A->n, nnz = A->nnz;
    const int64_t nsl = (n + 63) / 64;
    if (n == 0) return reject("empty matrix");
    try {
        std::vector<int32_t> rp((size_t)n + 1), cl((size_t)std::max<int64_t>(nnz, 1));
        APCG_HIP(hipSetDevice(A->device));
        g_counters.d2h_copies += 2;
        APCG_HIP(hipMemcpy(rp.data(), A->rowptr, sizeof(int32_t) * ((size_t)n + 1), hipMemcpyDeviceToHost));
        if (nnz > 0) APCG_HIP(hipMemcpy(cl.data(), A->col, sizeof(int32_t) * (size_t)nnz, hipMemcpyDeviceToHost));
        std::vector<int32_t> offs;
        auto slice_offsets = [&](int64_t sl) {  // sorted distinct column offsets of slice sl
            offs.clear();
            for (int64_t i = sl * 64; i < std::min<int64_t>(n, sl * 64 + 64); ++i)
                for (int64_t e = rp[i]; e < rp[i + 1]; ++e) offs.push_back(cl[e] - (int32_t)i);
            std::sort(offs.begin(), offs.end());
            offs.erase(std::unique(offs.begin(), offs.end()), offs.end());
        };
        for (int64_t i = 0; i < n; ++i)
            for (int64_t e = rp[i] + 1; e < rp[i + 1]; ++e)
                if (cl[e] <= cl[e - 1]) return reject("a row's columns are not strictly increasing");
        int32_t U = 0;
        for (int64_t sl = 0; sl < nsl; ++sl) {
            slice_offsets(sl);
            if (offs.size() > 32) return reject("a slice has more than 32 distinct column offsets");
            U = std::max<int32_t>(U, (int32_t)offs.size());
        }
        U = std::max<int32_t>(U, 1);
        const int64_t slots = nsl * U * 64;
        const int64_t sell_bytes = 12 * (A->sell_entries >= 0 ? A->sell_entries : nnz);
        if (8 * slots > sell_bytes) return reject("the padded value copy would exceed the sliced copy");
        const int32_t MP = U <= 8 ? 8 : U <= 16 ? 16 : 32;
        // plane stride for marching: the largest offset o = 64 Ps (Ps < 65536)
        // present with both signs in at least half of the slices
        std::map<int32_t, int64_t> both;
        for (int64_t sl = 0; sl < nsl; ++sl) {
            slice_offsets(sl);
            for (int32_t o : offs)
                if (o > 0 && o % 64 == 0 && o / 64 < 65536 && std::binary_search(offs.begin(), offs.end(), -o)) ++both[o];
        }
        int32_t ps = 0;
        for (auto &kv : both)
            if (2 * kv.second >= nsl) ps = kv.first / 64;
        // offsets, then the partner slots, then the value-symmetry flag
        std::vector<int32_t> off_h((size_t)(2 * nsl * MP + 64), 0);
        std::vector<uint64_t> msk_h((size_t)(nsl * MP), 0);
        for (int64_t sl = 0; sl < nsl; ++sl) {
            slice_offsets(sl);
            for (size_t k = 0; k < offs.size(); ++k) off_h[sl * MP + k] = offs[k];
            for (int64_t i = sl * 64; i < std::min<int64_t>(n, sl * 64 + 64); ++i)
                for (int64_t e = rp[i]; e < rp[i + 1]; ++e) {
                    const int64_t k = std::lower_bound(offs.begin(), offs.end(), cl[e] - (int32_t)i) - offs.begin();
                    msk_h[sl * MP + k] |= 1ull << (i - sl * 64);
                }
        }
        // Structural symmetry: every entry (i, j) has its transpose (j, i).
        // Then entry (i, i - q) of slice s, lane l is the transpose of entry
        // (i - q, i), which sits in the slot of offset +q of slice
        // (i - q) >> 6: slice s - q/64 for lanes l >= q mod 64, the slice
        // before it for the lanes below.  Those two slot indices are kept per
        // lower slot (low byte: upper lanes, next byte: lower lanes).
        bool sym = true;
        for (int64_t i = 0; i < n && sym; ++i)
            for (int64_t e = rp[i]; e < rp[i + 1]; ++e) {
                const int32_t j = cl[e];
                if (j < 0 || j >= n || !std::binary_search(cl.begin() + rp[j], cl.begin() + rp[j + 1], (int32_t)i)) {
                    sym = false;
                    break;
                }
            }
        int32_t *part_h = off_h.data() + nsl * MP;
        if (sym) {
            auto slot_of = [&](int64_t sl, int32_t o) -> int32_t {  // slot of offset o in slice sl, 0 if absent
                if (sl < 0) return 0;
                for (int32_t k = 0; k < MP; ++k)
                    if (off_h[sl * MP + k] == o) return k;
                return 0;
            };
            for (int64_t sl = 0; sl < nsl; ++sl)
                for (int32_t k = 0; k < MP; ++k) {
                    const int32_t o = off_h[sl * MP + k];
                    if (msk_h[sl * MP + k] == 0 || o >= 0) continue;
                    const int32_t q = -o, qs = q >> 6, qr = q & 63;
                    part_h[sl * MP + k] = slot_of(sl - qs, q) | (qr ? slot_of(sl - qs - 1, q) << 8 : 0);
                }
        }
        A->sdia_sym = sym ? 1 : 0;
        off_h[2 * nsl * MP] = A->sdia_sym;  // the value-symmetry flag, cleared by the check at a mismatch
        APCG_HIP(hipMalloc((void **)&A->sdia_off, sizeof(int32_t) * off_h.size()));
        APCG_HIP(hipMalloc((void **)&A->sdia_msk, sizeof(uint64_t) * nsl * MP));
        APCG_HIP(hipMalloc((void **)&A->sdia_val, sizeof(double) * slots));
        g_counters.h2d_copies += 2;
        APCG_HIP(hipMemcpy(A->sdia_off, off_h.data(), sizeof(int32_t) * off_h.size(), hipMemcpyHostToDevice));
        APCG_HIP(hipMemcpy(A->sdia_msk, msk_h.data(), sizeof(uint64_t) * nsl * MP, hipMemcpyHostToDevice));
        A->sdia_u = U;
        A->sdia_mp = MP;
        A->sdia_ps = ps;
        A->sdia_state = 1;
        return APCG_SUCCESS;
    } catch (const std::bad_alloc &) {
        return set_error(APCG_ERR_OUT_OF_MEMORY, "host allocation failed");
    }
}

// Queues the refill of the sliced-diagonal values from the CSR values on
// stream s (analysing the pattern first if needed).
apcg_status prepare_sdia(apcg_mat_s *A, hipStream_t s) {
    apcg_status st = sdia_analyse(A);
    if (st) return st;
    if (A->sdia_state < 0) return set_error(APCG_ERR_UNSUPPORTED, A->sdia_reason);
    const int64_t nsl = ((int64_t)A->n + 63) / 64;
    const int64_t blocks = (nsl * 64 + 255) / 256;
    int32_t *flag = A->sdia_off + 2 * nsl * A->sdia_mp;
    hipLaunchKernelGGL(k_sdia_fill, dim3((unsigned)blocks), dim3(256), 0, s, A->n, A->rowptr, A->val,
                       (const uint64_t *)A->sdia_msk, A->sdia_u, A->sdia_mp, A->sdia_val);
    APCG_CHECK_LAUNCH("k_sdia_fill");
    if (A->sdia_sym) {
        hipLaunchKernelGGL(k_sdia_symcheck, dim3((unsigned)blocks), dim3(256), 0, s, A->n, A->sdia_off,
                           (const uint64_t *)A->sdia_msk, A->sdia_u, A->sdia_mp, A->sdia_val, flag);
        APCG_CHECK_LAUNCH("k_sdia_symcheck");
    }
    return APCG_SUCCESS;
}

// Finds the matrix's distinct column offsets on the host from a copy of the
// CSR pattern (once per matrix) and allocates the diagonal copy and its
// table.  Leaves dia_state -1 with a reason when the layout does not apply.
apcg_status dia_analyse(apcg_mat_s *A) {
    if (A->dia_state != 0) return APCG_SUCCESS;
    auto reject = [&](const char *why) {
        A->dia_state = -1;
        A->dia_reason = why;
        return APCG_SUCCESS;
    };
    const int64_t n = A->n, nnz = A->nnz;
    if (n == 0) return reject("empty matrix");
    try {
        std::vector<int32_t> rp((size_t)n + 1), cl((size_t)std::max<int64_t>(nnz, 1));
        APCG_HIP(hipSetDevice(A->device));
        g_counters.d2h_copies += 2;
        APCG_HIP(hipMemcpy(rp.data(), A->rowptr, sizeof(int32_t) * ((size_t)n + 1), hipMemcpyDeviceToHost));
        if (nnz > 0) APCG_HIP(hipMemcpy(cl.data(), A->col, sizeof(int32_t) * (size_t)nnz, hipMemcpyDeviceToHost));
        std::vector<int32_t> offs;  // sorted distinct offsets
        for (int64_t i = 0; i < n; ++i)
            for (int64_t e = rp[i]; e < rp[i + 1]; ++e) {
                if (e > rp[i] && cl[e] <= cl[e - 1]) return reject("a row's columns are not strictly increasing");
                const int32_t o = cl[e] - (int32_t)i;
                auto it = std::lower_bound(offs.begin(), offs.end(), o);
                if (it == offs.end() || *it != o) {
                    if ((int)offs.size() == kDiaMaxDiags) return reject("more than 9 distinct column offsets");
                    offs.insert(it, o);
                }
            }
        if (offs.empty()) return reject("no entries");
        const int nd = (int)offs.size();
        const int ndt = nd <= 5 ? 5 : nd <= 7 ? 7 : 9;
        int32_t tab[32];
        for (int k = 0; k < 32; ++k) tab[k] = 0;
        bool sym = true;
        for (int k = 0; k < kDiaMaxDiags; ++k) {
            tab[k] = k < nd ? offs[k] : 0;
            tab[9 + k] = -1;
            if (k < nd) {
                auto it = std::lower_bound(offs.begin(), offs.end(), -offs[k]);
                const bool has = it != offs.end() && *it == -offs[k];
                if (!has) sym = false;
                if (offs[k] < 0 && has) tab[9 + k] = (int32_t)(it - offs.begin());
            }
        }
        tab[18] = sym ? 1 : 0;
        tab[19] = nd;
        // plane stride for marching: the largest offset 64 Ps (Ps < 65536)
        // present with both signs
        int32_t ps = 0;
        for (int k = 0; k < nd; ++k) {
            const int32_t o = offs[k];
            if (o > 0 && o % 64 == 0 && o / 64 < 65536 && std::binary_search(offs.begin(), offs.end(), -o))
                ps = std::max<int32_t>(ps, o / 64);
        }
        const int64_t stride = (n + 63) / 64 * 64;
        APCG_HIP(hipMalloc((void **)&A->dia_tab, sizeof(tab)));
        APCG_HIP(hipMalloc((void **)&A->dia_val, sizeof(double) * ndt * stride));
        g_counters.h2d_copies++;
        APCG_HIP(hipMemcpy(A->dia_tab, tab, sizeof(tab), hipMemcpyHostToDevice));
        for (int k = 0; k < kDiaMaxDiags; ++k) A->dia_off_h[k] = tab[k];
        A->dia_nd = nd;
        A->dia_ndt = ndt;
        A->dia_sym = sym ? 1 : 0;
        A->dia_ps = ps;
        A->dia_state = 1;
        return APCG_SUCCESS;
    } catch (const std::bad_alloc &) {
        return set_error(APCG_ERR_OUT_OF_MEMORY, "host allocation failed");
    }
}

// Queues the refill of the diagonals from the CSR values on stream s (and
// the value-symmetry check when the offset set is symmetric).
apcg_status prepare_dia(apcg_mat_s *A, hipStream_t s) {
    apcg_status st = dia_analyse(A);
    if (st) return st;
    if (A->dia_state < 0) return set_error(APCG_ERR_UNSUPPORTED, A->dia_reason);
    const int64_t stride = ((int64_t)A->n + 63) / 64 * 64;
    hipLaunchKernelGGL(k_dia_fill, dim3((unsigned)((stride + 255) / 256)), dim3(256), 0, s, A->n, A->rowptr,
                       A->col, A->val, (const int32_t *)A->dia_tab, A->dia_ndt, A->dia_val);
    APCG_CHECK_LAUNCH("k_dia_fill");
    if (A->dia_sym) {
        hipLaunchKernelGGL(k_dia_symcheck, dim3((unsigned)(((int64_t)A->n + 255) / 256)), dim3(256), 0, s, A->n,
                           A->dia_tab, (const double *)A->dia_val);
        APCG_CHECK_LAUNCH("k_dia_symcheck");
    }
    return APCG_SUCCESS;
}

namespace {

struct Bufs {
    const apcg_mat_s *A;
    double *x;
    const double *b;
    Workspace ws;
    double *partials;
    double *part_res() const { return partials + (size_t)kSliceResidual * kMaxBlocks; }
    double *part_delta() const { return partials + (size_t)kSliceDelta * kMaxBlocks; }
};

apcg_status launch_product(hipStream_t s, const Plan &pl, const Bufs &bf, int iter, int tune = 0) {
    const double *pold = bf.ws.p((iter + 1) & 1);
    double *pnew = bf.ws.p(iter & 1);
    hipLaunchKernelGGL(pl.prod, dim3(pl.g_prod), dim3(pl.tb), pl.lds_bytes, s, pl.n, pl.a0, pl.a1, pl.a2,
                       (const double *)bf.ws.z(), pold, pnew, bf.ws.w(),
                       bf.ws.state, (const double *)bf.part_res(), pl.g_vec, bf.part_delta(), pl.rpb, iter & 1, tune,
                       pl.lds_nnz);
    APCG_CHECK_LAUNCH("k_pcg_product");
    return APCG_SUCCESS;
}

apcg_status launch_update(hipStream_t s, const Plan &pl, const Bufs &bf, int iter, int norm_pre, int tune = 0) {
    const double *p = bf.ws.p(iter & 1);
    hipLaunchKernelGGL(k_pcg_update, dim3(pl.g_vec), dim3(VB), 0, s, (int64_t)pl.n, bf.x, bf.ws.r(), p,
                       (const double *)bf.ws.w(), (const double *)bf.ws.dinv(), bf.ws.z(), bf.ws.state,
                       (const double *)bf.part_delta(), pl.g_prod, bf.part_res(), pl.pb_vec, iter & 1, norm_pre,
                       tune);
    APCG_CHECK_LAUNCH("k_pcg_update");
    return APCG_SUCCESS;
}

apcg_status get_graph(apcg_ctx c, const Plan &pl, const Bufs &bf, int K, int pc, int norm_pre,
                      hipGraphExec_t *exec) {
    GraphKey key;
    key.mat_uid = bf.A->uid;
    key.rowptr = pl.a0;
    key.col = pl.a1;
    key.val = pl.a2;
    key.x = bf.x;
    key.ws = bf.ws.base;
    key.state = bf.ws.state;
    key.partials = bf.partials;
    key.prod = reinterpret_cast<const void *>(pl.prod);
    key.ws_cap = bf.ws.cap;
    key.pb_vec = pl.pb_vec;
    key.lds_bytes = (int64_t)pl.lds_bytes;
    key.n = pl.n;
    key.K = K;
    key.tb = pl.tb;
    key.g_prod = pl.g_prod;
    key.rpb = pl.rpb;
    key.g_vec = pl.g_vec;
    key.lds_nnz = pl.lds_nnz;
    key.pc = pc;
    key.norm = norm_pre;
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
    return apcg::pcg_solve_marked(ctx, A, b, x, rtol, maxit, opts_in, info, info_index, nullptr, 0);
}

}  // extern "C"

namespace apcg {

apcg_status pcg_solve_marked(apcg_ctx ctx, apcg_mat A, apcg_vec b, apcg_vec x, double rtol, int32_t maxit,
                             const apcg_solve_opts *opts_in, apcg_info info, int32_t info_index, double *hist,
                             int32_t hist_cap, const int32_t *gate) {
    try {
        if (!A || !b || !x || !info) return set_error(APCG_ERR_INVALID_ARG, "NULL argument");
        if (b->n != A->n || x->n != A->n) return set_error(APCG_ERR_INVALID_ARG, "dimension mismatch");
        if (vec_overlap(b, x)) return set_error(APCG_ERR_INVALID_ARG, "b and x must not share memory");
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
        if (opts.mode < APCG_MODE_GRAPH || opts.mode > APCG_MODE_AUTO)
            return set_error(APCG_ERR_INVALID_ARG, "unknown mode");
        if (opts.mode == APCG_MODE_AUTO)
            opts.mode = A->n <= APCG_PERSISTENT_MAX_N && !hist && !gate && !opts.kernel_timing ? APCG_MODE_PERSISTENT
                                                                                              : APCG_MODE_GRAPH;
        if (opts.mode == APCG_MODE_PERSISTENT && (A->n > APCG_PERSISTENT_MAX_N || hist || gate))
            return set_error(APCG_ERR_INVALID_ARG, "the persistent mode takes n <= APCG_PERSISTENT_MAX_N");
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
        const int norm_pre = opts.norm_type == APCG_NORM_PRECONDITIONED;
        hipStream_t st = c->stream;
        if (opts.mode == APCG_MODE_PERSISTENT) {  // reads the CSR arrays; p in the workspace
            if ((s = launch_pcg_wg(st, A->n, A->rowptr, A->col, A->val, b->d, x->d, c->ws.p(0), rtol, maxit,
                                   opts.x0_is_zero ? 1 : 0, opts.pc, norm_pre, A->sell_maxw, info->d + info_index)))
                return s;
            return op_end(c, acc, 4);
        }
        if (A->cfg.schedule == APCG_SPMV_SELL && (s = prepare_sell(A, c->stream))) return s;
        if (A->cfg.schedule == APCG_SPMV_SDIA && (s = prepare_sdia(A, c->stream))) return s;
        if (A->cfg.schedule == APCG_SPMV_DIA && (s = prepare_dia(A, c->stream))) return s;
        Plan pl;
        if ((s = make_plan(A, A->cfg, &pl))) return s;
        Bufs bf{A, x->d, b->d, c->ws, c->partials};

        hipLaunchKernelGGL(k_pcg_init, dim3(pl.g_vec), dim3(VB), 0, st, A->n, A->rowptr, A->col, A->val, b->d, x->d,
                           c->ws.r(), c->ws.dinv(), c->ws.z(), c->ws.p(0), bf.part_res(), pl.pb_vec,
                           opts.x0_is_zero ? 1 : 0, opts.pc, norm_pre, gate);
        APCG_CHECK_LAUNCH("k_pcg_init");
        hipLaunchKernelGGL(k_pcg_init_final, dim3(1), dim3(64), 0, st, c->ws.state, (const double *)bf.part_res(),
                           pl.g_vec, rtol, maxit, hist, hist_cap, gate);
        APCG_CHECK_LAUNCH("k_pcg_init_final");
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
                        g_counters.host_polls++;
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
                            g_counters.host_polls++;
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
                    if (done) break;
                    if ((s = launch_update(st, pl, bf, k, norm_pre))) return s;
                    if ((s = queue_poll(c, bf, 0))) return s;
                    g_counters.host_syncs++;
                    if ((s = check_poll(c, 0, &done))) return s;
                    if (done) break;
                }
            }
        }
        hipLaunchKernelGGL(k_pcg_finish, dim3(1), dim3(64), 0, st, c->ws.state, (const double *)bf.part_res(),
                           pl.g_vec, info->d + info_index);
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

}  // namespace apcg

extern "C" {

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
        if (ctx->tkind[2 * i] != kind || ctx->tkind[2 * i + 1] > hs.out_its) continue;
        float ms = 0.f;
        APCG_HIP(hipEventElapsedTime(&ms, ctx->tev[2 * i], ctx->tev[2 * i + 1]));
        total += ms;
        ++n;
    }
    *count = n;
    *mean_us = n ? 1000.0 * total / n : 0.0;
    return APCG_SUCCESS;
}

apcg_status apcg_mat_time_kernels(apcg_mat A, apcg_ctx ctx, int32_t reps, double *product_us, double *update_us) {
    try {
        if (!A || !ctx || reps < 1 || !product_us || !update_us)
            return set_error(APCG_ERR_INVALID_ARG, "bad timing arguments");
        if (ctx->device != A->device) return set_error(APCG_ERR_INVALID_ARG, "operands on different devices");
        if (ctx->type == APCG_STREAM_GLOBAL_BLOCKING)
            return set_error(APCG_ERR_INVALID_ARG, "kernel timing needs a default-stream context");
        Acc acc[1] = {{&A->rec, ACC_R}};
        apcg_status s;
        if ((s = op_begin(ctx, acc, 1))) return s;
        if ((s = ensure_workspace(ctx, A->n))) return s;
        hipStream_t st = ctx->stream;
        const int64_t n = A->n;
        hipLaunchKernelGGL(k_tune_fill, dim3(1024), dim3(VB), 0, st, ctx->ws.r(), ctx->ws.dinv(), ctx->ws.p(0),
                           ctx->ws.z(), n);
        APCG_CHECK_LAUNCH("k_tune_fill");
        if (A->cfg.schedule == APCG_SPMV_SELL && (s = prepare_sell(A, st))) return s;
        if (A->cfg.schedule == APCG_SPMV_SDIA && (s = prepare_sdia(A, st))) return s;
        if (A->cfg.schedule == APCG_SPMV_DIA && (s = prepare_dia(A, st))) return s;
        Plan pl;
        if ((s = make_plan(A, A->cfg, &pl))) return s;
        double *xs = nullptr;  // stand-in for x: the timed update writes it
        APCG_HIP(hipMalloc((void **)&xs, sizeof(double) * std::max<int64_t>(n, 1)));
        APCG_HIP(hipMemsetAsync(xs, 0, sizeof(double) * std::max<int64_t>(n, 1), st));
        Bufs bf{A, xs, nullptr, ctx->ws, ctx->partials};
        hipEvent_t ev[3];
        for (auto &e : ev) APCG_HIP(hipEventCreate(&e));
        for (int w = 0; w < 2; ++w) {
            if ((s = launch_product(st, pl, bf, 1, 1))) return s;
            if ((s = launch_update(st, pl, bf, 1, 0, 1))) return s;
        }
        APCG_HIP(hipEventRecord(ev[0], st));
        for (int r = 0; r < reps; ++r)
            if ((s = launch_product(st, pl, bf, 1, 1))) return s;
        APCG_HIP(hipEventRecord(ev[1], st));
        for (int r = 0; r < reps; ++r)
            if ((s = launch_update(st, pl, bf, 1, 0, 1))) return s;
        APCG_HIP(hipEventRecord(ev[2], st));
        g_counters.host_syncs++;
        APCG_HIP(hipEventSynchronize(ev[2]));
        float m0 = 0.f, m1 = 0.f;
        APCG_HIP(hipEventElapsedTime(&m0, ev[0], ev[1]));
        APCG_HIP(hipEventElapsedTime(&m1, ev[1], ev[2]));
        for (auto &e : ev) hipEventDestroy(e);
        hipFree(xs);  // the stream is idle here (synchronised on the last event)
        *product_us = 1000.0 * m0 / reps;
        *update_us = 1000.0 * m1 / reps;
        return op_end(ctx, acc, 1);
    } catch (const std::bad_alloc &) {
        return set_error(APCG_ERR_OUT_OF_MEMORY, "host allocation failed");
    }
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
        hipLaunchKernelGGL(k_tune_fill, dim3(1024), dim3(VB), 0, st, ctx->ws.r(), ctx->ws.dinv(), ctx->ws.p(0),
                           ctx->ws.z(), n);
        APCG_CHECK_LAUNCH("k_tune_fill");
        double *xs = nullptr;  // stand-in for x: the tuned update writes it
        APCG_HIP(hipMalloc((void **)&xs, sizeof(double) * std::max<int64_t>(n, 1)));
        APCG_HIP(hipMemsetAsync(xs, 0, sizeof(double) * std::max<int64_t>(n, 1), st));
        Bufs bf{A, xs, nullptr, ctx->ws, ctx->partials};
        const double per_row = n > 0 ? (double)A->nnz / n : 1.0;
        hipEvent_t e0, e1;
        APCG_HIP(hipEventCreate(&e0));
        APCG_HIP(hipEventCreate(&e1));
        double best_t = 1e300;
        apcg_spmv_config best_cfg = A->cfg;
        const bool sell_ok = A->sell_entries >= 0;
        if (sell_ok && (s = prepare_sell(A, st))) return s;
        if ((s = sdia_analyse(A))) return s;
        const bool sdia_ok = A->sdia_state == 1;
        if (sdia_ok && (s = prepare_sdia(A, st))) return s;
        if ((s = dia_analyse(A))) return s;
        const bool dia_ok = A->dia_state == 1;
        if (dia_ok && (s = prepare_dia(A, st))) return s;
        // -4: diagonals, -2: sliced diagonals, -1: the sliced schedule, 0:
        // the staged one, -3 / -5: sliced diagonals / diagonals with plane
        // marching (the inner value is the number of planes per task, not a
        // grid)
        // one product + update pair per repetition, both with their partial
        // reductions, after two untimed pairs
        auto time_pair = [&](const Plan &pl, double *us) -> apcg_status {
            apcg_status ts;
            for (int w = 0; w < 2; ++w) {
                if ((ts = launch_product(st, pl, bf, 1, 1))) return ts;
                if ((ts = launch_update(st, pl, bf, 1, 0, 1))) return ts;
            }
            APCG_HIP(hipEventRecord(e0, st));
            for (int r = 0; r < reps; ++r) {
                if ((ts = launch_product(st, pl, bf, 1, 1))) return ts;
                if ((ts = launch_update(st, pl, bf, 1, 0, 1))) return ts;
            }
            APCG_HIP(hipEventRecord(e1, st));
            g_counters.host_syncs++;
            APCG_HIP(hipEventSynchronize(e1));
            float ms = 0.f;
            APCG_HIP(hipEventElapsedTime(&ms, e0, e1));
            *us = 1000.0 * ms / reps;
            return APCG_SUCCESS;
        };
        std::vector<std::pair<double, apcg_spmv_config>> timed;
        for (int lpr : {-5, -4, -3, -2, -1, 0, 1, 2, 4, 8, 16, 32, 64}) {
            if (lpr > 1 && lpr > 4 * std::max(1.0, per_row)) continue;
            if (lpr == -4 && !dia_ok) continue;
            if (lpr == -5 && !(dia_ok && A->dia_ps > 0)) continue;
            if (lpr == -1 && !sell_ok) continue;
            if (lpr == -2 && !sdia_ok) continue;
            if (lpr == -3 && !(sdia_ok && A->sdia_ps > 0)) continue;
            for (int tb : {256, 512}) {
                if (lpr == 0 && !stream_fits(A, tb)) continue;
                // marching: planes per task (how many tasks fill the resident
                // wavefronts depends on the grid's plane count); otherwise
                // the grid size
                static const int kGrids[] = {256, 512, 1024, 2048, 4096, 8192};
                static const int kPlanes[] = {4, 6, 8};
                const bool march = lpr == -3 || lpr == -5;
                const int *inner = march ? kPlanes : kGrids;
                const int ninner = march ? 3 : 6;
                for (int q = 0; q < ninner; ++q) {
                    const int blocks = inner[q], seg = inner[q];
                    apcg_spmv_config cfg = lpr == -5  ? apcg_spmv_config{seg, tb, 0, APCG_SPMV_DIA}
                                           : lpr == -4 ? apcg_spmv_config{1, tb, blocks, APCG_SPMV_DIA}
                                           : lpr == -3 ? apcg_spmv_config{seg, tb, 0, APCG_SPMV_SDIA}
                                           : lpr == -2 ? apcg_spmv_config{1, tb, blocks, APCG_SPMV_SDIA}
                                           : lpr == -1 ? apcg_spmv_config{1, tb, blocks, APCG_SPMV_SELL}
                                           : lpr == 0 ? apcg_spmv_config{1, tb, blocks, APCG_SPMV_STREAM}
                                                      : apcg_spmv_config{lpr, tb, blocks, APCG_SPMV_ROWGROUP};
                    Plan pl;
                    if ((s = make_plan(A, cfg, &pl))) return s;
                    if (!march && pl.g_prod < blocks && blocks > 256) continue;  // same grid as a smaller one
                    double us;
                    if ((s = time_pair(pl, &us))) return s;
                    timed.push_back({us, cfg});
                }
            }
        }
        // the four fastest timed twice more, in turn, each keeping its best
        // time: a single window can be disturbed (clocks, other work)
        std::sort(timed.begin(), timed.end(),
                  [](const std::pair<double, apcg_spmv_config> &a, const std::pair<double, apcg_spmv_config> &b) {
                      return a.first < b.first;
                  });
        if (timed.size() > 4) timed.resize(4);
        for (int pass = 0; pass < 2; ++pass)
            for (auto &tc : timed) {
                Plan pl;
                if ((s = make_plan(A, tc.second, &pl))) return s;
                double us;
                if ((s = time_pair(pl, &us))) return s;
                tc.first = std::min(tc.first, us);
            }
        for (const auto &tc : timed)
            if (tc.first < best_t) {
                best_t = tc.first;
                best_cfg = tc.second;
            }
        hipEventDestroy(e0);
        hipEventDestroy(e1);
        hipFree(xs);  // the stream is idle here (synchronised on the last timing event)
        A->cfg = best_cfg;
        if (best) *best = best_cfg;
        if (best_us) *best_us = best_t;
        return op_end(ctx, acc, 1);
    } catch (const std::bad_alloc &) {
        return set_error(APCG_ERR_OUT_OF_MEMORY, "host allocation failed");
    }
}

}  // extern "C"
