// tune.hip -- the autotuner's results, kept and reused.
//
// The product schedule the autotuner picks (apcg_mat_autotune: timed on the
// device) depends on the device and on the shape of the matrix far more than
// on its values.  Results are therefore kept in a table keyed by
//
//   <arch> | <pattern class> | n<floor(log2 n)> | r<round(4 nnz / n)>
//
// where the pattern class names what decides which schedules apply and how
// they behave:
//   u<U>   the most distinct column offsets (column - row) in any 64-row
//          slice, capped at 33 (the sliced-diagonal layout takes U <= 32);
//   d<D>   the distinct offsets of the whole matrix when there are at most
//          9 (the diagonal layout), else 0;
//   p<0|1> an offset 64 P present with both signs in at least half of the
//          slices (plane marching applies);
//   s<0|1> the pattern is structurally symmetric (transposed value reads);
//   m<M>   the longest row.
// The table lives in host memory for the process; apcg_tune_cache_load and
// apcg_tune_cache_save read and write it as text, one entry per line
// (key, four integers, microseconds; tab separated), so a later process --
// or the next run on the same kind of device -- skips the timing sweep.
// Batched solves keep their tuned configurations in the same table under
// keys that start with "batch|".
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "internal.h"

namespace apcg {

namespace {

struct TuneVal {
    int32_t v[4];
    double us;
};

std::mutex g_tune_mu;
std::map<std::string, TuneVal> g_tune;
std::map<int, std::string> g_arch;  // gcnArchName per device

}  // namespace

std::string pattern_class(int64_t n, int64_t nnz, const int32_t *rp, const int32_t *cl) {
    (void)nnz;
    int64_t maxrow = 0;
    for (int64_t i = 0; i < n; ++i) maxrow = std::max<int64_t>(maxrow, rp[i + 1] - rp[i]);
    // distinct offsets: per slice, and over the whole matrix (up to 10 kept)
    const int64_t nsl = (n + 63) / 64;
    std::vector<int32_t> offs, all;
    bool many = false;
    int64_t U = 0;
    std::map<int32_t, int64_t> both;  // offset 64 P present with both signs: slice count
    for (int64_t sl = 0; sl < nsl; ++sl) {
        offs.clear();
        for (int64_t i = sl * 64; i < std::min<int64_t>(n, sl * 64 + 64); ++i)
            for (int64_t e = rp[i]; e < rp[i + 1]; ++e) offs.push_back(cl[e] - (int32_t)i);
        std::sort(offs.begin(), offs.end());
        offs.erase(std::unique(offs.begin(), offs.end()), offs.end());
        U = std::max<int64_t>(U, (int64_t)offs.size());
        for (int32_t o : offs) {
            if (o > 0 && o % 64 == 0 && o / 64 < 65536 && std::binary_search(offs.begin(), offs.end(), -o)) ++both[o];
            if (!many) {
                auto it = std::lower_bound(all.begin(), all.end(), o);
                if (it == all.end() || *it != o) {
                    if (all.size() == 9) many = true;
                    else all.insert(it, o);
                }
            }
        }
    }
    bool plane = false;
    for (auto &kv : both)
        if (2 * kv.second >= nsl) plane = true;
    bool sym = true;
    for (int64_t i = 0; i < n && sym; ++i)
        for (int64_t e = rp[i]; e < rp[i + 1]; ++e) {
            const int32_t j = cl[e];
            if (j < 0 || j >= n || !std::binary_search(cl + rp[j], cl + rp[j + 1], (int32_t)i)) {
                sym = false;
                break;
            }
        }
    char buf[96];
    snprintf(buf, sizeof buf, "u%d.d%d.p%d.s%d.m%lld", (int)std::min<int64_t>(U, 33), many ? 0 : (int)all.size(),
             plane ? 1 : 0, sym ? 1 : 0, (long long)maxrow);
    return buf;
}

std::string tune_key(const std::string &arch, const std::string &cls, int64_t n, int64_t nnz) {
    int lg = 0;
    while (lg < 62 && ((int64_t)1 << (lg + 1)) <= n) ++lg;
    const long long r4 = n > 0 ? llround(4.0 * (double)nnz / (double)n) : 0;
    return arch + "|" + cls + "|n" + std::to_string(lg) + "|r" + std::to_string(r4);
}

apcg_status device_arch(int device, std::string *out) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_arch.find(device);
    if (it == g_arch.end()) {
        hipDeviceProp_t p;
        APCG_HIP(hipGetDeviceProperties(&p, device));
        it = g_arch.emplace(device, std::string(p.gcnArchName)).first;
    }
    *out = it->second;
    return APCG_SUCCESS;
}

// The tuning key of matrix A (its pattern read back once and the class kept
// with the matrix).
apcg_status mat_tune_key(apcg_mat_s *A, std::string *key) {
    if (A->tune_class.empty()) {
        const int64_t n = A->n, nnz = A->nnz;
        std::vector<int32_t> rp((size_t)n + 1), cl((size_t)std::max<int64_t>(nnz, 1));
        APCG_HIP(hipSetDevice(A->device));
        g_counters.d2h_copies += 2;
        APCG_HIP(hipMemcpy(rp.data(), A->rowptr, sizeof(int32_t) * ((size_t)n + 1), hipMemcpyDeviceToHost));
        if (nnz > 0) APCG_HIP(hipMemcpy(cl.data(), A->col, sizeof(int32_t) * (size_t)nnz, hipMemcpyDeviceToHost));
        A->tune_class = pattern_class(n, nnz, rp.data(), cl.data());
    }
    std::string arch;
    apcg_status s;
    if ((s = device_arch(A->device, &arch))) return s;
    *key = tune_key(arch, A->tune_class, A->n, A->nnz);
    return APCG_SUCCESS;
}

bool tune_lookup(const std::string &key, int32_t v[4], double *us) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune.find(key);
    if (it == g_tune.end()) return false;
    memcpy(v, it->second.v, sizeof it->second.v);
    if (us) *us = it->second.us;
    return true;
}

void tune_insert(const std::string &key, const int32_t v[4], double us) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    TuneVal t;
    memcpy(t.v, v, sizeof t.v);
    t.us = us;
    g_tune[key] = t;
}

}  // namespace apcg

using namespace apcg;

namespace {

apcg_status copy_key(const std::string &key, char *out, int32_t cap) {
    if (!out || cap < 1) return set_error(APCG_ERR_INVALID_ARG, "no room for the key");
    if ((int64_t)key.size() + 1 > cap) return set_error(APCG_ERR_INVALID_ARG, "key buffer too small");
    memcpy(out, key.c_str(), key.size() + 1);
    return APCG_SUCCESS;
}

bool key_ok(const char *key) {
    if (!key || !*key) return false;
    for (const char *c = key; *c; ++c)
        if (*c == '\t' || *c == '\n' || *c == '\r') return false;
    return true;
}

}  // namespace

extern "C" {

apcg_status apcg_tune_key_pattern(const char *arch, int32_t n, int64_t nnz, const int32_t *rowptr,
                                  const int32_t *col, char *out, int32_t cap) {
    try {
        if (!arch || !key_ok(arch) || n < 0 || nnz < 0 || (!rowptr && n > 0) || (!col && nnz > 0))
            return set_error(APCG_ERR_INVALID_ARG, "bad pattern arguments");
        if (n > 0 && (rowptr[0] != 0 || rowptr[n] != nnz))
            return set_error(APCG_ERR_INVALID_ARG, "rowptr does not span nnz");
        for (int32_t i = 0; i < n; ++i)
            if (rowptr[i + 1] < rowptr[i]) return set_error(APCG_ERR_INVALID_ARG, "rowptr is decreasing");
        return copy_key(tune_key(arch, pattern_class(n, nnz, rowptr, col), n, nnz), out, cap);
    } catch (const std::bad_alloc &) {
        return set_error(APCG_ERR_OUT_OF_MEMORY, "host allocation failed");
    }
}

apcg_status apcg_mat_tune_key(apcg_mat A, char *out, int32_t cap) {
    try {
        if (!A) return set_error(APCG_ERR_INVALID_ARG, "matrix is NULL");
        std::string key;
        apcg_status s;
        if ((s = mat_tune_key(A, &key))) return s;
        return copy_key(key, out, cap);
    } catch (const std::bad_alloc &) {
        return set_error(APCG_ERR_OUT_OF_MEMORY, "host allocation failed");
    }
}

apcg_status apcg_tune_cache_insert(const char *key, const int32_t values[4], double us) {
    try {
        if (!key_ok(key) || !values) return set_error(APCG_ERR_INVALID_ARG, "bad cache entry");
        tune_insert(key, values, us);
        return APCG_SUCCESS;
    } catch (const std::bad_alloc &) {
        return set_error(APCG_ERR_OUT_OF_MEMORY, "host allocation failed");
    }
}

apcg_status apcg_tune_cache_lookup(const char *key, int32_t values[4], double *us, int32_t *found) {
    try {
        if (!key_ok(key) || !values || !found) return set_error(APCG_ERR_INVALID_ARG, "bad lookup arguments");
        *found = tune_lookup(key, values, us) ? 1 : 0;
        return APCG_SUCCESS;
    } catch (const std::bad_alloc &) {
        return set_error(APCG_ERR_OUT_OF_MEMORY, "host allocation failed");
    }
}

apcg_status apcg_tune_cache_clear(void) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune.clear();
    return APCG_SUCCESS;
}

apcg_status apcg_tune_cache_size(int32_t *entries) {
    if (!entries) return set_error(APCG_ERR_INVALID_ARG, "NULL argument");
    std::lock_guard<std::mutex> lk(g_tune_mu);
    *entries = (int32_t)g_tune.size();
    return APCG_SUCCESS;
}

apcg_status apcg_tune_cache_load(const char *path, int32_t *entries) {
    try {
        if (!path) return set_error(APCG_ERR_INVALID_ARG, "path is NULL");
        FILE *f = fopen(path, "r");
        if (!f) return set_error(APCG_ERR_INVALID_ARG, std::string("cannot open tuning cache ") + path);
        std::vector<std::pair<std::string, TuneVal>> got;
        char line[1024];
        int lineno = 0;
        bool bad = false;
        while (fgets(line, sizeof line, f)) {
            ++lineno;
            size_t len = strlen(line);
            while (len && (line[len - 1] == '\n' || line[len - 1] == '\r')) line[--len] = 0;
            if (!len || line[0] == '#') continue;
            char *tab = strchr(line, '\t');
            if (!tab) {
                bad = true;
                break;
            }
            *tab = 0;
            TuneVal t;
            if (sscanf(tab + 1, "%d %d %d %d\t%lf", &t.v[0], &t.v[1], &t.v[2], &t.v[3], &t.us) != 5 ||
                !key_ok(line)) {
                bad = true;
                break;
            }
            got.emplace_back(line, t);
        }
        fclose(f);
        if (bad)
            return set_error(APCG_ERR_INVALID_ARG,
                             std::string("malformed tuning cache line ") + std::to_string(lineno) + " in " + path);
        std::lock_guard<std::mutex> lk(g_tune_mu);
        for (auto &e : got) g_tune[e.first] = e.second;
        if (entries) *entries = (int32_t)got.size();
        return APCG_SUCCESS;
    } catch (const std::bad_alloc &) {
        return set_error(APCG_ERR_OUT_OF_MEMORY, "host allocation failed");
    }
}

apcg_status apcg_tune_cache_save(const char *path, int32_t *entries) {
    try {
        if (!path) return set_error(APCG_ERR_INVALID_ARG, "path is NULL");
        std::map<std::string, TuneVal> snap;
        {
            std::lock_guard<std::mutex> lk(g_tune_mu);
            snap = g_tune;
        }
        const std::string tmp = std::string(path) + ".tmp";
        FILE *f = fopen(tmp.c_str(), "w");
        if (!f) return set_error(APCG_ERR_INVALID_ARG, std::string("cannot write tuning cache ") + tmp);
        fprintf(f, "# key\tfour integers\tmicroseconds (autotuner results)\n");
        for (auto &e : snap)
            fprintf(f, "%s\t%d %d %d %d\t%.17g\n", e.first.c_str(), e.second.v[0], e.second.v[1], e.second.v[2],
                    e.second.v[3], e.second.us);
        const bool ok = fclose(f) == 0;
        if (!ok || rename(tmp.c_str(), path) != 0)
            return set_error(APCG_ERR_INVALID_ARG, std::string("cannot write tuning cache ") + path);
        if (entries) *entries = (int32_t)snap.size();
        return APCG_SUCCESS;
    } catch (const std::bad_alloc &) {
        return set_error(APCG_ERR_OUT_OF_MEMORY, "host allocation failed");
    }
}

apcg_status apcg_mat_autotune_cached(apcg_mat A, apcg_ctx ctx, int32_t reps, apcg_spmv_config *best,
                                     double *best_us, int32_t *from_cache) {
    try {
        if (!A || !ctx || reps < 1) return set_error(APCG_ERR_INVALID_ARG, "bad autotune arguments");
        std::string key;
        apcg_status s;
        if ((s = mat_tune_key(A, &key))) return s;
        int32_t v[4];
        double us = 0.0;
        if (tune_lookup(key, v, &us)) {
            const apcg_spmv_config cfg{v[0], v[1], v[2], v[3]};
            // applied only if this matrix takes it (the analyses it needs
            // succeed); otherwise tuned afresh
            if (apcg_mat_set_spmv_config(A, &cfg) == APCG_SUCCESS) {
                if (best) *best = cfg;
                if (best_us) *best_us = us;
                if (from_cache) *from_cache = 1;
                return APCG_SUCCESS;
            }
        }
        apcg_spmv_config cfg;
        if ((s = apcg_mat_autotune(A, ctx, reps, &cfg, &us))) return s;
        const int32_t nv[4] = {cfg.lanes_per_row, cfg.block_size, cfg.blocks, cfg.schedule};
        tune_insert(key, nv, us);
        if (best) *best = cfg;
        if (best_us) *best_us = us;
        if (from_cache) *from_cache = 0;
        return APCG_SUCCESS;
    } catch (const std::bad_alloc &) {
        return set_error(APCG_ERR_OUT_OF_MEMORY, "host allocation failed");
    }
}

}  // extern "C"
