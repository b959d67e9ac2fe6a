// learn.hip -- the learned part of the polynomial preconditioner.
//
//   * features of one system: row statistics of A, Gershgorin bounds of
//     D^-1 A, and the Ritz values of the Lanczos tridiagonal that 12
//     Jacobi-PCG iterations build (the CG-Lanczos relation; the iterations
//     run on the solve kernels, the tridiagonal's eigenvalues by Sturm-count
//     bisection, one thread per eigenvalue);
//   * the training label of one system: the smallest Ritz value lmin of its
//     full Jacobi-PCG solve (Sturm-sequence multisection on the tridiagonal
//     of all iterations), a = 3 lmin clamped to [1e-3 lmax, lmax / 2], and
//     the target p* = the Chebyshev semi-iterative polynomial on [a, lmax]
//     (its residual polynomial is the minimax one there), as the quadratic
//     form (G, h) of the loss;
//   * a 16 -> 64 -> 64 -> 9 tanh MLP in FP32: forward, loss, backward,
//     Adam, all with fixed reduction orders (deterministic).
//
// The polynomial is p(t) = sum_j c_j T_j(2 t / lmax - 1) on [0, lmax],
// lmax = the Gershgorin upper bound of D^-1 A.  Loss of one system:
//   L(c) = c'G c - 2 h'c + 1 + mu/Q sum_q max(0, eps - p(s_q))^2
// with G = G0 / kappa, h = G0 c* / kappa, kappa = c*' G0 c*,
// G0_jk = sum_q w_q t_q^2 T_j(y_q) T_k(y_q) over the 16-point Gauss-Chebyshev
// rule (t_q on [a, lmax], w_q = 1/16, y_q = 2 t_q / lmax - 1): the relative
// mean-square distance of the residual polynomial 1 - t p(t) from the
// minimax one, plus a positivity penalty on Q = 64 points s_q of [0, lmax].
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>

#include "internal.h"

namespace apcg {
namespace {

constexpr int FB = 256;   // block size of the row-statistics kernels
constexpr int MSTEPS = 12;
constexpr int NF = 16, NH = 64, NC = 9, NPARAM = 5833, QGRID = 64;
constexpr int LABEL_Q = 16;
constexpr double LABEL_SHIFT = 3.0;
constexpr double LABEL_FLOOR = 1e-3;  // keeps the target's minimum away from zero
constexpr int OFF_W1 = 0, OFF_B1 = 1024, OFF_W2 = 1088, OFF_B2 = 5184, OFF_W3 = 5248, OFF_B3 = 5824;

// Row statistics, pass 1 -> partials [7][G] (dev::RowStats order).
__global__ __launch_bounds__(FB) void k_feat_rows(int32_t n, const int32_t *__restrict__ rowptr,
                                                  const int32_t *__restrict__ col, const double *__restrict__ val,
                                                  double *part, int64_t per_block) {
    const dev::Chunk c = dev::block_chunk(n, per_block);
    dev::RowStats a;
    for (int64_t i = c.lo + threadIdx.x; i < c.hi; i += FB) dev::row_stats_add(a, rowptr, col, val, i);
    __shared__ double sh[7][FB];
    dev::row_stats_block<FB>(a, sh);
    if (threadIdx.x == 0) {
        const int lb = dev::xcd_block(blockIdx.x, gridDim.x);
        for (int k = 0; k < 7; ++k) part[k * gridDim.x + lb] = a.v[k];
    }
}

// One workgroup of FB: pass-1 totals -> stats[0..6] (stats[7] = mean ln d);
// thread t merges partials t, t + FB, ..., then the fixed tree.
__global__ __launch_bounds__(FB) void k_feat_rows_final(const double *part, int G, int32_t n, double *stats) {
    dev::RowStats a;
    for (int g = threadIdx.x; g < G; g += FB) {
        double b[7];
        for (int k = 0; k < 7; ++k) b[k] = part[k * G + g];
        dev::row_stats_merge(a, b);
    }
    __shared__ double sh[7][FB];
    dev::row_stats_block<FB>(a, sh);
    if (threadIdx.x != 0) return;
    for (int k = 0; k < 7; ++k) stats[k] = a.v[k];
    stats[7] = a.v[4] / (double)n;
}

// Pass 2: partials of sum (ln d_i - mean)^2 (two-pass variance).
__global__ __launch_bounds__(FB) void k_feat_rows2(int32_t n, const int32_t *__restrict__ rowptr,
                                                   const int32_t *__restrict__ col, const double *__restrict__ val,
                                                   const double *stats, double *part, int64_t per_block) {
    const dev::Chunk c = dev::block_chunk(n, per_block);
    const double mean = stats[7];
    double acc = 0.0;
    for (int64_t i = c.lo + threadIdx.x; i < c.hi; i += FB) {
        const double e = dev::row_logdiag(rowptr, col, val, i) - mean;
        acc = fma(e, e, acc);
    }
    double v[1] = {acc};
    dev::store_partials<FB, 1>(v, part, gridDim.x, dev::xcd_block(blockIdx.x, gridDim.x));
}

__device__ double cheb(int j, double y) {  // T_j(y) by the recurrence, any real y
    double t0 = 1.0, t1 = y;
    if (j == 0) return t0;
    for (int k = 2; k <= j; ++k) {
        const double t2 = 2.0 * y * t1 - t0;
        t0 = t1;
        t1 = t2;
    }
    return t1;
}

// One workgroup of 64: thread i < m finds the i-th smallest Ritz value (the
// eigenvalues of the 12-step Lanczos tridiagonal); thread 0 then forms the
// 16 features (FP32) and lmax (FP64).
__global__ __launch_bounds__(64) void k_feat_final(const double *stats, const double *var_part, int Gv,
                                                   const double *hist, int hist_cap, const apcg_solve_info *info,
                                                   int32_t n, int64_t nnz, float *feat, double *lmax_out) {
    int m = info->iterations;
    if (m > hist_cap) m = hist_cap;
    if (m > 16) m = 16;
    const double *al = hist, *be = hist + hist_cap;
    __shared__ double th[16], td[16], te2[16];
    dev::ritz_values(al, be, m, td, te2, th);
    double vs[1];
    dev::reduce_partials<64, 1>(var_part, Gv, vs);  // sum of squared deviations, fixed order
    __syncthreads();
    if (threadIdx.x != 0) return;
    if (m < 1) {  // no iteration (b = 0): lmax stands in as the only Ritz value
        th[0] = stats[1];
        m = 1;
    }
    const double var = vs[0];
    const double relres = info->ref_norm > 0.0 ? info->res_norm / info->ref_norm : 1.0;
    dev::feature_vector(stats, var, th, m, relres, n, nnz, feat);
    *lmax_out = stats[1];
}

// One workgroup of 64: the smallest eigenvalue by multisection (each round
// splits the bracket into 65 parts and keeps the one where the count first
// reaches 1), then the interval, the target's coefficients (interpolation at
// the 9 Chebyshev points, exact for a degree-8 polynomial:
// c_j = (2 - [j = 0]) / 9 sum_k p*(t(y_k)) T_j(y_k), y_k = cos(pi (k + 1/2) / 9))
// and the loss's normalised quadratic form.
__global__ __launch_bounds__(64) void k_label(const double *stats, const double *hist, int cap,
                                              const apcg_solve_info *info, float *Gout, float *hout,
                                              double *lab) {
    const double hi = stats[1];
    int m = info->iterations;
    if (m > cap) m = cap;
    const double *al = hist, *be = hist + cap;
    __shared__ double s_lo, s_hi;
    __shared__ int first;
    if (threadIdx.x == 0) {
        s_lo = -0.5 * hi;
        s_hi = 1.5 * hi;
    }
    __syncthreads();
    if (m > 0) {
        for (int round = 0; round < 10; ++round) {
            const double lo = s_lo, w = (s_hi - lo) / 65.0;
            const double x = lo + w * (threadIdx.x + 1);
            const bool hit = dev::sturm_below(al, be, m, x) >= 1;
            if (threadIdx.x == 0) first = 64;
            __syncthreads();
            if (hit) atomicMin(&first, (int)threadIdx.x);
            __syncthreads();
            if (threadIdx.x == 0) {
                const int f = first;
                s_lo = lo + w * f;  // count(lo + w f) == 0 (f = 0: the old lower end)
                if (f < 64) s_hi = lo + w * (f + 1);
            }
            __syncthreads();
        }
    }
    if (threadIdx.x != 0) return;
    const double lmin = m > 0 ? 0.5 * (s_lo + s_hi) : 0.0;
    double a = 0.5 * hi;
    if (m > 0) a = fmin(fmax(LABEL_SHIFT * lmin, LABEL_FLOOR * hi), 0.5 * hi);
    // target coefficients
    const double s0 = (hi + a) / (hi - a), T9s0 = cheb(9, s0);
    double cs[NC];
    for (int j = 0; j < NC; ++j) cs[j] = 0.0;
    for (int k = 0; k < NC; ++k) {
        const double y = cos(M_PI * (k + 0.5) / NC);
        const double t = 0.5 * (y + 1.0) * hi;
        const double pv = (1.0 - cheb(9, (hi + a - 2.0 * t) / (hi - a)) / T9s0) / t;
        for (int j = 0; j < NC; ++j) cs[j] += pv * cheb(j, y);
    }
    for (int j = 0; j < NC; ++j) cs[j] *= (j == 0 ? 1.0 : 2.0) / NC;
    // G0 over the Gauss-Chebyshev rule on [a, hi]
    double G[NC][NC];
    for (int j = 0; j < NC; ++j)
        for (int k = 0; k < NC; ++k) G[j][k] = 0.0;
    for (int q = 0; q < LABEL_Q; ++q) {
        const double t = 0.5 * (a + hi) + 0.5 * (hi - a) * cos((2 * q + 1) * M_PI / (2 * LABEL_Q));
        const double y = 2.0 * t / hi - 1.0, w = 1.0 / LABEL_Q;
        double T[NC];
        T[0] = 1.0;
        T[1] = y;
        for (int j = 2; j < NC; ++j) T[j] = 2.0 * y * T[j - 1] - T[j - 2];
        for (int j = 0; j < NC; ++j)
            for (int k = 0; k < NC; ++k) G[j][k] += w * t * t * T[j] * T[k];
    }
    double Gc[NC], kappa = 0.0;
    for (int j = 0; j < NC; ++j) {
        Gc[j] = 0.0;
        for (int k = 0; k < NC; ++k) Gc[j] += G[j][k] * cs[k];
        kappa += cs[j] * Gc[j];
    }
    for (int j = 0; j < NC; ++j) {
        hout[j] = (float)(Gc[j] / kappa);
        for (int k = 0; k < NC; ++k) Gout[j * NC + k] = (float)(G[j][k] / kappa);
    }
    lab[0] = lmin;
    lab[1] = a;
    lab[2] = hi;
}

// ----------------------------------------------------------------- MLP
__global__ void k_phi_grid(float *phi) {
    const int q = threadIdx.x;  // Q = 64 threads
    if (q >= QGRID) return;
    const double y = -1.0 + 2.0 * q / (QGRID - 1);
    for (int j = 0; j < NC; ++j) phi[q * NC + j] = (float)cheb(j, y);
}

// One workgroup of 64 threads per sample.
__global__ __launch_bounds__(64) void k_mlp_fwd(const float *__restrict__ P, const float *__restrict__ X, int B,
                                                float *__restrict__ H1, float *__restrict__ H2,
                                                float *__restrict__ C) {
    const int b = blockIdx.x, j = threadIdx.x;
    if (b >= B) return;
    __shared__ float x[NF], h1[NH], h2[NH];
    if (j < NF) x[j] = X[b * NF + j];
    __syncthreads();
    float a = P[OFF_B1 + j];
    for (int k = 0; k < NF; ++k) a = fmaf(P[OFF_W1 + j * NF + k], x[k], a);
    const float t1 = tanhf(a);
    h1[j] = t1;
    if (H1) H1[b * NH + j] = t1;
    __syncthreads();
    a = P[OFF_B2 + j];
    for (int k = 0; k < NH; ++k) a = fmaf(P[OFF_W2 + j * NH + k], h1[k], a);
    const float t2 = tanhf(a);
    h2[j] = t2;
    if (H2) H2[b * NH + j] = t2;
    __syncthreads();
    if (j < NC) {
        a = P[OFF_B3 + j];
        for (int k = 0; k < NH; ++k) a = fmaf(P[OFF_W3 + j * NH + k], h2[k], a);
        C[b * NC + j] = a;
    }
}

// Per-sample loss and dL/dc (already divided by B for the mean loss).
__global__ __launch_bounds__(64) void k_mlp_loss(const float *__restrict__ C, const float *__restrict__ G,
                                                 const float *__restrict__ h, const float *__restrict__ phi, int B,
                                                 float mu, float eps, float *__restrict__ dC,
                                                 float *__restrict__ loss_b) {
    const int b = blockIdx.x, t = threadIdx.x;
    if (b >= B) return;
    __shared__ float c[NC], viol[QGRID];
    if (t < NC) c[t] = C[b * NC + t];
    __syncthreads();
    float q = 0.f;
    for (int j = 0; j < NC; ++j) q = fmaf(phi[t * NC + j], c[j], q);
    viol[t] = fmaxf(0.f, eps - q);
    __syncthreads();
    const float scale = mu / (float)QGRID;
    if (t < NC) {
        float g = -2.f * h[b * NC + t];
        for (int k = 0; k < NC; ++k) g = fmaf(2.f * G[b * NC * NC + t * NC + k], c[k], g);
        float pen = 0.f;
        for (int qq = 0; qq < QGRID; ++qq) pen = fmaf(viol[qq], phi[qq * NC + t], pen);
        g = fmaf(-2.f * scale, pen, g);
        dC[b * NC + t] = g / (float)B;
    }
    if (t == 0) {
        float L = 1.f;
        for (int j = 0; j < NC; ++j) {
            float gc = 0.f;
            for (int k = 0; k < NC; ++k) gc = fmaf(G[b * NC * NC + j * NC + k], c[k], gc);
            L = fmaf(c[j], gc - 2.f * h[b * NC + j], L);
        }
        float pen = 0.f;
        for (int qq = 0; qq < QGRID; ++qq) pen = fmaf(viol[qq], viol[qq], pen);
        loss_b[b] = fmaf(scale, pen, L);
    }
}

// Per-sample back-propagated activation gradients dA2 = (dC W3) (1 - h2^2),
// dA1 = (dA2 W2) (1 - h1^2).
__global__ __launch_bounds__(64) void k_mlp_bwd_act(const float *__restrict__ P, const float *__restrict__ dC,
                                                    const float *__restrict__ H1, const float *__restrict__ H2, int B,
                                                    float *__restrict__ dA1, float *__restrict__ dA2) {
    const int b = blockIdx.x, j = threadIdx.x;
    if (b >= B) return;
    __shared__ float dc[NC], da2[NH];
    if (j < NC) dc[j] = dC[b * NC + j];
    __syncthreads();
    float a = 0.f;
    for (int o = 0; o < NC; ++o) a = fmaf(dc[o], P[OFF_W3 + o * NH + j], a);
    const float h2 = H2[b * NH + j];
    const float d2 = a * (1.f - h2 * h2);
    da2[j] = d2;
    dA2[b * NH + j] = d2;
    __syncthreads();
    a = 0.f;
    for (int k = 0; k < NH; ++k) a = fmaf(da2[k], P[OFF_W2 + k * NH + j], a);
    const float h1 = H1[b * NH + j];
    dA1[b * NH + j] = a * (1.f - h1 * h1);
}

// Parameter gradients: one thread per parameter, sum over samples in order.
__global__ __launch_bounds__(256) void k_mlp_grad(const float *__restrict__ X, const float *__restrict__ H1,
                                                  const float *__restrict__ H2, const float *__restrict__ dC,
                                                  const float *__restrict__ dA1, const float *__restrict__ dA2, int B,
                                                  float *__restrict__ grad) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= NPARAM) return;
    float g = 0.f;
    if (p < OFF_B1) {
        const int j = p / NF, k = p % NF;
        for (int b = 0; b < B; ++b) g = fmaf(dA1[b * NH + j], X[b * NF + k], g);
    } else if (p < OFF_W2) {
        const int j = p - OFF_B1;
        for (int b = 0; b < B; ++b) g += dA1[b * NH + j];
    } else if (p < OFF_B2) {
        const int j = (p - OFF_W2) / NH, k = (p - OFF_W2) % NH;
        for (int b = 0; b < B; ++b) g = fmaf(dA2[b * NH + j], H1[b * NH + k], g);
    } else if (p < OFF_W3) {
        const int j = p - OFF_B2;
        for (int b = 0; b < B; ++b) g += dA2[b * NH + j];
    } else if (p < OFF_B3) {
        const int o = (p - OFF_W3) / NH, k = (p - OFF_W3) % NH;
        for (int b = 0; b < B; ++b) g = fmaf(dC[b * NC + o], H2[b * NH + k], g);
    } else {
        const int o = p - OFF_B3;
        for (int b = 0; b < B; ++b) g += dC[b * NC + o];
    }
    grad[p] = g;
}

__global__ __launch_bounds__(256) void k_adam(float *__restrict__ P, const float *__restrict__ g,
                                              float *__restrict__ m, float *__restrict__ v, int t, float lr, float b1,
                                              float b2, float eps) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= NPARAM) return;
    const float gi = g[p];
    const float mi = b1 * m[p] + (1.f - b1) * gi;
    const float vi = b2 * v[p] + (1.f - b2) * gi * gi;
    m[p] = mi;
    v[p] = vi;
    const float mh = mi / (1.f - powf(b1, (float)t));
    const float vh = vi / (1.f - powf(b2, (float)t));
    P[p] -= lr * mh / (sqrtf(vh) + eps);
}

__global__ void k_loss_mean(const float *loss_b, int B, float *out) {
    if (threadIdx.x != 0) return;
    double s = 0.0;
    for (int b = 0; b < B; ++b) s += loss_b[b];
    *out = (float)(s / B);
}

// Column statistics (two-pass) and in-place standardisation of X [B, 16].
__global__ void k_standardize(float *X, int B, float *mean, float *stdv, int compute) {
    const int f = threadIdx.x;
    if (f >= NF) return;
    if (compute) {
        double s = 0.0;
        for (int b = 0; b < B; ++b) s += X[b * NF + f];
        const double mu = s / B;
        double q = 0.0;
        for (int b = 0; b < B; ++b) {
            const double e = X[b * NF + f] - mu;
            q += e * e;
        }
        const double sd = sqrt(q / B);
        mean[f] = (float)mu;
        stdv[f] = (float)(sd > 1e-12 ? sd : 1.0);
    }
    const float mu = mean[f], sd = stdv[f];
    for (int b = 0; b < B; ++b) X[b * NF + f] = (X[b * NF + f] - mu) / sd;
}

// Per-context MLP scratch (activations and gradients for up to cap samples).
struct MlpScratch {
    int device = 0;
    int64_t cap = 0;
    float *buf = nullptr;  // H1, H2, C, dC, dA1, dA2, loss_b, grad, phi
    float *H1() const { return buf; }
    float *H2() const { return buf + cap * NH; }
    float *C() const { return buf + 2 * cap * NH; }
    float *dC() const { return buf + 2 * cap * NH + cap * NC; }
    float *dA1() const { return buf + 2 * cap * NH + 2 * cap * NC; }
    float *dA2() const { return buf + 3 * cap * NH + 2 * cap * NC; }
    float *loss_b() const { return buf + 4 * cap * NH + 2 * cap * NC; }
    float *grad() const { return buf + 4 * cap * NH + 2 * cap * NC + cap; }
    float *phi() const { return grad() + NPARAM; }
    static size_t floats(int64_t cap) { return (size_t)(4 * cap * NH + 2 * cap * NC + cap + NPARAM + QGRID * NC); }
};

struct FeatScratch {
    int device = 0;
    int64_t cap = 0;
    double *x = nullptr;      // n doubles
    double *stats = nullptr;  // 8 + partials
    double *hist = nullptr;   // 2 * MSTEPS
    double *lhist = nullptr;  // 2 * lhist_cap: alpha, beta of a full solve
    int64_t lhist_cap = 0;
    float *fbuf = nullptr;    // learned solve: features [16], coefficients [9]
    double *dbuf = nullptr;   // learned solve: lmax
    apcg_info info = nullptr;
};

}  // namespace

static std::mutex g_learn_mu;
static std::vector<std::pair<uint64_t, MlpScratch *>> g_mlp;
static std::vector<std::pair<uint64_t, FeatScratch *>> g_feat;

static MlpScratch *mlp_scratch(apcg_ctx c) {
    std::lock_guard<std::mutex> lk(g_learn_mu);
    for (auto &p : g_mlp)
        if (p.first == c->id) return p.second;
    MlpScratch *s = new MlpScratch();
    s->device = c->device;
    g_mlp.emplace_back(c->id, s);
    return s;
}

static FeatScratch *feat_scratch(apcg_ctx c) {
    std::lock_guard<std::mutex> lk(g_learn_mu);
    for (auto &p : g_feat)
        if (p.first == c->id) return p.second;
    FeatScratch *s = new FeatScratch();
    s->device = c->device;
    g_feat.emplace_back(c->id, s);
    return s;
}

void learn_cache_release(uint64_t ctx_id, int device) {
    MlpScratch *m = nullptr;
    FeatScratch *f = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_learn_mu);
        for (auto it = g_mlp.begin(); it != g_mlp.end(); ++it)
            if (it->first == ctx_id) {
                m = it->second;
                g_mlp.erase(it);
                break;
            }
        for (auto it = g_feat.begin(); it != g_feat.end(); ++it)
            if (it->first == ctx_id) {
                f = it->second;
                g_feat.erase(it);
                break;
            }
    }
    hipSetDevice(device);
    if (m) {
        hipFree(m->buf);
        delete m;
    }
    if (f) {
        hipFree(f->x);
        hipFree(f->stats);
        hipFree(f->hist);
        hipFree(f->lhist);
        hipFree(f->fbuf);
        hipFree(f->dbuf);
        if (f->info) apcg_info_destroy(f->info);
        delete f;
    }
}

static apcg_status ensure_mlp(apcg_ctx c, MlpScratch *s, int64_t B) {
    if (s->buf && s->cap >= B) return APCG_SUCCESS;
    if (s->buf) {
        EventRef ev = event_get(c->device);
        if (!ev) return set_error(APCG_ERR_HIP, "event creation failed");
        APCG_HIP(hipEventRecord(ev->e, c->stream));
        float *old = s->buf;
        const int dev = c->device;
        defer_release({ev}, [old, dev]() {
            hipSetDevice(dev);
            hipFree(old);
        });
        s->buf = nullptr;
    }
    const int64_t cap = std::max<int64_t>(B, 256);
    APCG_HIP(hipMalloc((void **)&s->buf, sizeof(float) * MlpScratch::floats(cap)));
    s->cap = cap;
    hipLaunchKernelGGL(k_phi_grid, dim3(1), dim3(64), 0, c->stream, s->phi());
    APCG_CHECK_LAUNCH("k_phi_grid");
    return APCG_SUCCESS;
}

apcg_status mlp_infer(apcg_ctx ctx, const float *params, const float *mean, const float *std, float *X, int32_t B,
                      float *C) {
    if (B < 1) return APCG_SUCCESS;
    hipLaunchKernelGGL(k_standardize, dim3(1), dim3(64), 0, ctx->stream, X, B, (float *)mean, (float *)std, 0);
    APCG_CHECK_LAUNCH("k_standardize");
    hipLaunchKernelGGL(k_mlp_fwd, dim3(B), dim3(64), 0, ctx->stream, params, (const float *)X, B, (float *)nullptr,
                       (float *)nullptr, C);
    APCG_CHECK_LAUNCH("k_mlp_fwd");
    return APCG_SUCCESS;
}

// Allocates the per-context feature scratch for n rows (ordered after the
// context's pending work when it grows).
static apcg_status feat_prepare(apcg_ctx ctx, FeatScratch *fs, int64_t n) {
    apcg_status s;
    if (!fs->stats) {
        APCG_HIP(hipMalloc((void **)&fs->stats, sizeof(double) * (8 + 8 * (int64_t)kMaxBlocks)));
        APCG_HIP(hipMalloc((void **)&fs->hist, sizeof(double) * 2 * MSTEPS));
        APCG_HIP(hipMalloc((void **)&fs->fbuf, sizeof(float) * 32));
        APCG_HIP(hipMalloc((void **)&fs->dbuf, sizeof(double) * 4));
        if ((s = apcg_info_create(ctx->device, 1, &fs->info))) return s;
    }
    if (fs->cap < n) {
        if (fs->x) {
            EventRef ev = event_get(ctx->device);
            if (!ev) return set_error(APCG_ERR_HIP, "event creation failed");
            APCG_HIP(hipEventRecord(ev->e, ctx->stream));
            double *old = fs->x;
            const int dev = ctx->device;
            defer_release({ev}, [old, dev]() {
                hipSetDevice(dev);
                hipFree(old);
            });
            fs->x = nullptr;
        }
        APCG_HIP(hipMalloc((void **)&fs->x, sizeof(double) * n));
        fs->cap = n;
    }
    return APCG_SUCCESS;
}

// Row statistics (both passes) into fs->stats; partials after the first 8.
static apcg_status feat_rows(apcg_ctx ctx, apcg_mat A, FeatScratch *fs, int *G_out) {
    hipStream_t st = ctx->stream;
    int G;
    int64_t pb;
    elementwise_grid(A->n, &G, &pb);
    double *part = fs->stats + 8;
    hipLaunchKernelGGL(k_feat_rows, dim3(G), dim3(FB), 0, st, A->n, A->rowptr, A->col, A->val, part, pb);
    APCG_CHECK_LAUNCH("k_feat_rows");
    hipLaunchKernelGGL(k_feat_rows_final, dim3(1), dim3(FB), 0, st, (const double *)part, G, A->n, fs->stats);
    APCG_CHECK_LAUNCH("k_feat_rows_final");
    hipLaunchKernelGGL(k_feat_rows2, dim3(G), dim3(FB), 0, st, A->n, A->rowptr, A->col, A->val,
                       (const double *)fs->stats, part, pb);
    APCG_CHECK_LAUNCH("k_feat_rows2");
    *G_out = G;
    return APCG_SUCCESS;
}

static apcg_status check_system(apcg_ctx ctx, apcg_mat A, apcg_vec b) {
    if (!ctx || !A || !b) return set_error(APCG_ERR_INVALID_ARG, "NULL argument");
    if (b->n != A->n || A->n < 1) return set_error(APCG_ERR_INVALID_ARG, "dimension mismatch or empty system");
    if (ctx->device != A->device || b->device != A->device)
        return set_error(APCG_ERR_INVALID_ARG, "operands on different devices");
    return APCG_SUCCESS;
}

// Features into dev_feat[16] / dev_lmax[1] (device pointers), on ctx.
static apcg_status features_into(apcg_ctx ctx, apcg_mat A, apcg_vec b, float *dev_feat, double *dev_lmax) {
    FeatScratch *fs = feat_scratch(ctx);
    apcg_status s;
    APCG_HIP(hipSetDevice(ctx->device));
    if ((s = feat_prepare(ctx, fs, A->n))) return s;
    // 12 Jacobi-PCG steps from x0 = 0 with rtol = 0 record alpha and beta
    apcg_vec_s xv;
    xv.device = ctx->device;
    xv.d = fs->x;
    xv.n = A->n;
    apcg_solve_opts o;
    apcg_solve_opts_default(&o);
    o.x0_is_zero = 1;
    o.iters_per_graph = MSTEPS;  // one captured period, cached per matrix like the solve's
    if ((s = pcg_solve_marked(ctx, A, b, &xv, 0.0, MSTEPS, &o, fs->info, 0, fs->hist, MSTEPS))) return s;
    Acc acc[2] = {{&A->rec, ACC_R}, {&b->rec, ACC_R}};
    if ((s = op_begin(ctx, acc, 2))) return s;
    int G;
    if ((s = feat_rows(ctx, A, fs, &G))) return s;
    hipLaunchKernelGGL(k_feat_final, dim3(1), dim3(64), 0, ctx->stream, (const double *)fs->stats,
                       (const double *)(fs->stats + 8), G, (const double *)fs->hist, MSTEPS,
                       (const apcg_solve_info *)fs->info->d, A->n, A->nnz, dev_feat, dev_lmax);
    APCG_CHECK_LAUNCH("k_feat_final");
    return op_end(ctx, acc, 2);
}

}  // namespace apcg

using namespace apcg;

extern "C" {

apcg_status apcg_pc_features(apcg_ctx ctx, apcg_mat A, apcg_vec b, float *dev_feat, double *dev_lmax) {
    try {
        apcg_status s;
        if ((s = check_system(ctx, A, b))) return s;
        if (!dev_feat || !dev_lmax) return set_error(APCG_ERR_INVALID_ARG, "NULL argument");
        return features_into(ctx, A, b, dev_feat, dev_lmax);
    } catch (const std::bad_alloc &) {
        return set_error(APCG_ERR_OUT_OF_MEMORY, "host allocation failed");
    }
}

apcg_status apcg_pc_label(apcg_ctx ctx, apcg_mat A, apcg_vec b, double rtol, int32_t maxit, float *dev_G,
                          float *dev_h, double *dev_label) {
    try {
        apcg_status s;
        if ((s = check_system(ctx, A, b))) return s;
        if (!dev_G || !dev_h || !dev_label) return set_error(APCG_ERR_INVALID_ARG, "NULL argument");
        if (maxit < 1) return set_error(APCG_ERR_INVALID_ARG, "maxit must be >= 1");
        FeatScratch *fs = feat_scratch(ctx);
        APCG_HIP(hipSetDevice(ctx->device));
        if ((s = feat_prepare(ctx, fs, A->n))) return s;
        if (fs->lhist_cap < maxit) {
            if (fs->lhist) {
                EventRef ev = event_get(ctx->device);
                if (!ev) return set_error(APCG_ERR_HIP, "event creation failed");
                APCG_HIP(hipEventRecord(ev->e, ctx->stream));
                double *old = fs->lhist;
                const int dev = ctx->device;
                defer_release({ev}, [old, dev]() {
                    hipSetDevice(dev);
                    hipFree(old);
                });
                fs->lhist = nullptr;
            }
            APCG_HIP(hipMalloc((void **)&fs->lhist, sizeof(double) * 2 * (int64_t)maxit));
            fs->lhist_cap = maxit;
        }
        const int cap = (int)fs->lhist_cap;
        apcg_vec_s xv;
        xv.device = ctx->device;
        xv.d = fs->x;
        xv.n = A->n;
        apcg_solve_opts o;
        apcg_solve_opts_default(&o);
        o.x0_is_zero = 1;
        if ((s = pcg_solve_marked(ctx, A, b, &xv, rtol, maxit, &o, fs->info, 0, fs->lhist, cap))) return s;
        Acc acc[2] = {{&A->rec, ACC_R}, {&b->rec, ACC_R}};
        if ((s = op_begin(ctx, acc, 2))) return s;
        int G;
        if ((s = feat_rows(ctx, A, fs, &G))) return s;
        hipLaunchKernelGGL(k_label, dim3(1), dim3(64), 0, ctx->stream, (const double *)fs->stats,
                           (const double *)fs->lhist, cap, (const apcg_solve_info *)fs->info->d, dev_G, dev_h,
                           dev_label);
        APCG_CHECK_LAUNCH("k_label");
        return op_end(ctx, acc, 2);
    } catch (const std::bad_alloc &) {
        return set_error(APCG_ERR_OUT_OF_MEMORY, "host allocation failed");
    }
}

apcg_status apcg_ksp_solve_learned(apcg_ctx ctx, apcg_mat A, apcg_vec b, apcg_vec x, double rtol, int32_t maxit,
                                   const float *dev_params, const float *dev_mean, const float *dev_std,
                                   const apcg_solve_opts *opts, const apcg_fcg_opts *fopts, apcg_info info,
                                   int32_t info_index) {
    try {
        apcg_status s;
        if ((s = check_system(ctx, A, b))) return s;
        if (!dev_params || !dev_mean || !dev_std) return set_error(APCG_ERR_INVALID_ARG, "NULL network argument");
        FeatScratch *fs = feat_scratch(ctx);
        APCG_HIP(hipSetDevice(ctx->device));
        if ((s = feat_prepare(ctx, fs, A->n))) return s;
        float *feat = fs->fbuf, *coef = fs->fbuf + NF;
        if ((s = features_into(ctx, A, b, feat, fs->dbuf))) return s;
        hipLaunchKernelGGL(k_standardize, dim3(1), dim3(64), 0, ctx->stream, feat, 1, (float *)dev_mean,
                           (float *)dev_std, 0);
        APCG_CHECK_LAUNCH("k_standardize");
        hipLaunchKernelGGL(k_mlp_fwd, dim3(1), dim3(64), 0, ctx->stream, dev_params, (const float *)feat, 1,
                           (float *)nullptr, (float *)nullptr, coef);
        APCG_CHECK_LAUNCH("k_mlp_fwd");
        apcg_solve_opts o;
        if (opts) o = *opts;
        else apcg_solve_opts_default(&o);
        if (o.x0_is_zero) {
            // Warm start: the feature run's Jacobi-PCG steps from x0 = 0 left
            // their iterate in the scratch x; the flexible solve continues
            // from it instead of discarding it.
            if (!x || x->n != A->n || x->device != A->device)
                return set_error(APCG_ERR_INVALID_ARG, "x does not match the system");
            Acc acc[1] = {{&x->rec, ACC_W}};
            if ((s = op_begin(ctx, acc, 1))) return s;
            APCG_HIP(hipMemcpyAsync(x->d, fs->x, sizeof(double) * (size_t)A->n, hipMemcpyDeviceToDevice,
                                    ctx->stream));
            if ((s = op_end(ctx, acc, 1))) return s;
            o.x0_is_zero = 0;
        }
        return apcg_ksp_solve_fcg_poly(ctx, A, b, x, rtol, maxit, coef, fs->dbuf, &o, fopts, info, info_index);
    } catch (const std::bad_alloc &) {
        return set_error(APCG_ERR_OUT_OF_MEMORY, "host allocation failed");
    }
}

apcg_status apcg_mlp_standardize(apcg_ctx ctx, float *dev_X, int32_t B, float *dev_mean, float *dev_std,
                                 int32_t compute_stats) {
    if (!ctx || !dev_X || !dev_mean || !dev_std || B < 1) return set_error(APCG_ERR_INVALID_ARG, "bad arguments");
    APCG_HIP(hipSetDevice(ctx->device));
    hipLaunchKernelGGL(k_standardize, dim3(1), dim3(64), 0, ctx->stream, dev_X, B, dev_mean, dev_std,
                       compute_stats ? 1 : 0);
    APCG_CHECK_LAUNCH("k_standardize");
    if (ctx->type == APCG_STREAM_GLOBAL_BLOCKING) APCG_HIP(hipStreamSynchronize(ctx->stream));
    return APCG_SUCCESS;
}

apcg_status apcg_mlp_forward(apcg_ctx ctx, const float *dev_params, const float *dev_X, int32_t B, float *dev_C) {
    if (!ctx || !dev_params || !dev_X || !dev_C || B < 1) return set_error(APCG_ERR_INVALID_ARG, "bad arguments");
    APCG_HIP(hipSetDevice(ctx->device));
    hipLaunchKernelGGL(k_mlp_fwd, dim3(B), dim3(64), 0, ctx->stream, dev_params, dev_X, B, (float *)nullptr,
                       (float *)nullptr, dev_C);
    APCG_CHECK_LAUNCH("k_mlp_fwd");
    if (ctx->type == APCG_STREAM_GLOBAL_BLOCKING) APCG_HIP(hipStreamSynchronize(ctx->stream));
    return APCG_SUCCESS;
}

apcg_status apcg_mlp_loss_grad(apcg_ctx ctx, const float *dev_params, const float *dev_X, const float *dev_G,
                               const float *dev_h, int32_t B, float mu, float eps, float *dev_loss,
                               float *dev_grad) {
    if (!ctx || !dev_params || !dev_X || !dev_G || !dev_h || !dev_loss || !dev_grad || B < 1)
        return set_error(APCG_ERR_INVALID_ARG, "bad arguments");
    APCG_HIP(hipSetDevice(ctx->device));
    MlpScratch *ms = mlp_scratch(ctx);
    apcg_status s;
    if ((s = ensure_mlp(ctx, ms, B))) return s;
    hipStream_t st = ctx->stream;
    hipLaunchKernelGGL(k_mlp_fwd, dim3(B), dim3(64), 0, st, dev_params, dev_X, B, ms->H1(), ms->H2(), ms->C());
    APCG_CHECK_LAUNCH("k_mlp_fwd");
    hipLaunchKernelGGL(k_mlp_loss, dim3(B), dim3(64), 0, st, (const float *)ms->C(), dev_G, dev_h,
                       (const float *)ms->phi(), B, mu, eps, ms->dC(), ms->loss_b());
    APCG_CHECK_LAUNCH("k_mlp_loss");
    hipLaunchKernelGGL(k_mlp_bwd_act, dim3(B), dim3(64), 0, st, dev_params, (const float *)ms->dC(),
                       (const float *)ms->H1(), (const float *)ms->H2(), B, ms->dA1(), ms->dA2());
    APCG_CHECK_LAUNCH("k_mlp_bwd_act");
    hipLaunchKernelGGL(k_mlp_grad, dim3((NPARAM + 255) / 256), dim3(256), 0, st, dev_X, (const float *)ms->H1(),
                       (const float *)ms->H2(), (const float *)ms->dC(), (const float *)ms->dA1(),
                       (const float *)ms->dA2(), B, dev_grad);
    APCG_CHECK_LAUNCH("k_mlp_grad");
    hipLaunchKernelGGL(k_loss_mean, dim3(1), dim3(64), 0, st, (const float *)ms->loss_b(), B, dev_loss);
    APCG_CHECK_LAUNCH("k_loss_mean");
    if (ctx->type == APCG_STREAM_GLOBAL_BLOCKING) APCG_HIP(hipStreamSynchronize(ctx->stream));
    return APCG_SUCCESS;
}

apcg_status apcg_mlp_train_step(apcg_ctx ctx, float *dev_params, float *dev_adam_m, float *dev_adam_v, int32_t t,
                                float lr, const float *dev_X, const float *dev_G, const float *dev_h, int32_t B,
                                float mu, float eps, float *dev_loss) {
    if (!dev_adam_m || !dev_adam_v || t < 1) return set_error(APCG_ERR_INVALID_ARG, "bad Adam state");
    MlpScratch *ms = mlp_scratch(ctx);
    apcg_status s;
    if ((s = ensure_mlp(ctx, ms, B))) return s;
    if ((s = apcg_mlp_loss_grad(ctx, dev_params, dev_X, dev_G, dev_h, B, mu, eps, dev_loss, ms->grad()))) return s;
    hipLaunchKernelGGL(k_adam, dim3((NPARAM + 255) / 256), dim3(256), 0, ctx->stream, dev_params,
                       (const float *)ms->grad(), dev_adam_m, dev_adam_v, t, lr, 0.9f, 0.999f, 1e-8f);
    APCG_CHECK_LAUNCH("k_adam");
    if (ctx->type == APCG_STREAM_GLOBAL_BLOCKING) APCG_HIP(hipStreamSynchronize(ctx->stream));
    return APCG_SUCCESS;
}

}  // extern "C"
