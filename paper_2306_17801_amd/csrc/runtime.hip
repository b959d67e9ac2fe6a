// runtime.hip -- execution contexts, the access registry, device scalars,
// vector/matrix wrappers, solve-info arrays, timers and diagnostics.
//
// The ordering model is the one of Section 3.1.2: an operation names the
// objects it reads and writes; on a different context than the previous
// user, a write waits for the last write and for every read since, and a read
// waits for the last write.  Reads are never ordered among themselves.  Waits
// are device-side (hipStreamWaitEvent); the host never blocks for ordering.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <deque>
#include <map>

#include "internal.h"

namespace apcg {

Counters g_counters;
std::recursive_mutex g_mu;

static thread_local std::string t_last_error;

apcg_status set_error(apcg_status code, const std::string &msg) {
    t_last_error = msg;
    return code;
}

apcg_status hip_error(hipError_t e, const char *what) {
    char buf[512];
    snprintf(buf, sizeof buf, "HIP error %d (%s) in %s", (int)e, hipGetErrorString(e), what);
    return set_error(e == hipErrorOutOfMemory ? APCG_ERR_OUT_OF_MEMORY : APCG_ERR_HIP, buf);
}

// ---------------------------------------------------------------------------
// event pool
// ---------------------------------------------------------------------------
static std::mutex g_ev_mu;
static std::map<int, std::vector<hipEvent_t>> g_ev_pool;

Event::~Event() {
    if (e) {
        std::lock_guard<std::mutex> lk(g_ev_mu);
        g_ev_pool[device].push_back(e);
    }
}

EventRef event_get(int device) {
    auto ev = std::make_shared<Event>();
    ev->device = device;
    {
        std::lock_guard<std::mutex> lk(g_ev_mu);
        auto &pool = g_ev_pool[device];
        if (!pool.empty()) {
            ev->e = pool.back();
            pool.pop_back();
        }
    }
    if (!ev->e) {
        int cur = 0;
        hipGetDevice(&cur);
        if (cur != device) hipSetDevice(device);
        if (hipEventCreateWithFlags(&ev->e, hipEventDisableTiming) != hipSuccess) ev->e = nullptr;
        if (cur != device) hipSetDevice(cur);
        if (!ev->e) return nullptr;
    }
    return ev;
}

static EventRef timing_event_get(int device) {
    auto ev = std::make_shared<Event>();
    ev->device = device;
    int cur = 0;
    hipGetDevice(&cur);
    if (cur != device) hipSetDevice(device);
    hipError_t e = hipEventCreate(&ev->e);
    if (cur != device) hipSetDevice(cur);
    if (e != hipSuccess) {
        ev->e = nullptr;
        return nullptr;
    }
    ev->device = -1 - device;  // timing events live in their own pool bucket
    return ev;
}

// ---------------------------------------------------------------------------
// deferred release
// ---------------------------------------------------------------------------
struct Deferred {
    std::vector<EventRef> deps;
    std::function<void()> fn;
};
static std::deque<Deferred> g_deferred;

void defer_release(std::vector<EventRef> deps, std::function<void()> fn) {
    std::lock_guard<std::recursive_mutex> lk(g_mu);
    g_deferred.push_back({std::move(deps), std::move(fn)});
}

void reap() {
    std::vector<std::function<void()>> ready;
    {
        std::lock_guard<std::recursive_mutex> lk(g_mu);
        for (auto it = g_deferred.begin(); it != g_deferred.end();) {
            bool done = true;
            for (auto &e : it->deps)
                if (e && e->e && hipEventQuery(e->e) == hipErrorNotReady) {
                    done = false;
                    break;
                }
            if (done) {
                ready.push_back(std::move(it->fn));
                it = g_deferred.erase(it);
            } else {
                ++it;
            }
        }
    }
    for (auto &f : ready) f();
}

std::vector<EventRef> record_deps(const Record &r) {
    std::vector<EventRef> d;
    if (r.write_ev) d.push_back(r.write_ev);
    for (auto &p : r.readers) d.push_back(p.second);
    return d;
}

// ---------------------------------------------------------------------------
// contexts
// ---------------------------------------------------------------------------
static std::atomic<uint64_t> g_next_id{1};
static std::map<int, apcg_ctx> g_default_ctx;  // per-device globally blocking ctx

static apcg_status ctx_init(apcg_ctx c, int32_t device, int32_t type) {
    c->id = g_next_id++;
    c->device = device;
    c->type = type;
    APCG_HIP(hipSetDevice(device));
    APCG_HIP(hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking));
    APCG_HIP(hipMalloc((void **)&c->partials, sizeof(double) * kPartialSlots * kMaxBlocks));
    APCG_HIP(hipHostMalloc((void **)&c->pinned_flags, sizeof(int32_t) * kMaxLookahead, hipHostMallocDefault));
    for (int i = 0; i < kMaxLookahead; ++i) c->pinned_flags[i] = 0;
    return APCG_SUCCESS;
}

static void ctx_release_now(apcg_ctx c) {
    hipSetDevice(c->device);
    batch_cache_release(c->id, c->device);
    seg_cache_release(c->id, c->device);
    learn_cache_release(c->id, c->device);
    fcg_cache_release(c->id, c->device);
    bfcg_cache_release(c->id, c->device);
    tq_cache_release(c->id, c->device);
    for (auto &g : c->graphs) {
        if (g.exec) hipGraphExecDestroy(g.exec);
        if (g.graph) hipGraphDestroy(g.graph);
    }
    for (auto e : c->tev) hipEventDestroy(e);
    if (c->ws.base) hipFree(c->ws.base);
    if (c->ws.state) hipFree(c->ws.state);
    if (c->partials) hipFree(c->partials);
    if (c->pinned_flags) hipHostFree(c->pinned_flags);
    if (c->stream) hipStreamDestroy(c->stream);
    delete c;
}

apcg_status resolve_ctx(apcg_ctx in, int device, apcg_ctx *out) {
    if (in) {
        if (in->device != device)
            return set_error(APCG_ERR_INVALID_ARG, "context and operands live on different devices");
        *out = in;
        return APCG_SUCCESS;
    }
    std::lock_guard<std::recursive_mutex> lk(g_mu);
    auto it = g_default_ctx.find(device);
    if (it != g_default_ctx.end()) {
        *out = it->second;
        return APCG_SUCCESS;
    }
    apcg_ctx c = new apcg_ctx_s();
    apcg_status st = ctx_init(c, device, APCG_STREAM_GLOBAL_BLOCKING);
    if (st != APCG_SUCCESS) {
        delete c;
        return st;
    }
    c->is_default_global = true;
    g_default_ctx[device] = c;
    *out = c;
    return APCG_SUCCESS;
}

// Marks the start of an operation of context c on the objects in acc:
// inserts the device-side waits the ordering rule requires.
apcg_status op_begin(apcg_ctx c, const Acc *acc, int n) {
    reap();
    APCG_HIP(hipSetDevice(c->device));
    if (c->type == APCG_STREAM_GLOBAL_BLOCKING) {
        // waits for all prior work of every stream on the device
        g_counters.host_syncs++;
        APCG_HIP(hipDeviceSynchronize());
        return APCG_SUCCESS;
    }
    std::lock_guard<std::recursive_mutex> lk(g_mu);
    std::vector<Event *> waited;
    auto wait = [&](const EventRef &e) -> apcg_status {
        if (!e || !e->e) return APCG_SUCCESS;
        if (std::find(waited.begin(), waited.end(), e.get()) != waited.end()) return APCG_SUCCESS;
        waited.push_back(e.get());
        g_counters.stream_waits++;
        APCG_HIP(hipStreamWaitEvent(c->stream, e->e, 0));
        return APCG_SUCCESS;
    };
    for (int i = 0; i < n; ++i) {
        Record *r = acc[i].rec;
        if (!r) continue;
        // a context that already read the object since its last write has
        // already waited for that write
        bool synced = false;
        for (auto &rd : r->readers)
            if (rd.first == c->id) synced = true;
        if (r->writer_ctx && r->writer_ctx != c->id && !synced) {
            apcg_status s = wait(r->write_ev);
            if (s) return s;
        }
        if (acc[i].mode & ACC_W) {
            for (auto &rd : r->readers)
                if (rd.first != c->id) {
                    apcg_status s = wait(rd.second);
                    if (s) return s;
                }
        }
    }
    return APCG_SUCCESS;
}

// Marks the end of the operation: one event records its completion and
// becomes the objects' last write or one of their reads.
apcg_status op_end(apcg_ctx c, const Acc *acc, int n) {
    EventRef ev = event_get(c->device);
    if (!ev) return set_error(APCG_ERR_HIP, "event creation failed");
    APCG_HIP(hipEventRecord(ev->e, c->stream));
    {
        std::lock_guard<std::recursive_mutex> lk(g_mu);
        for (int i = 0; i < n; ++i) {
            Record *r = acc[i].rec;
            if (!r) continue;
            if (acc[i].mode & ACC_W) {
                r->writer_ctx = c->id;
                r->write_ev = ev;
                r->readers.clear();
            } else {
                bool found = false;
                for (auto &rd : r->readers)
                    if (rd.first == c->id) {
                        rd.second = ev;
                        found = true;
                    }
                if (!found) r->readers.emplace_back(c->id, ev);
            }
        }
    }
    if (c->type == APCG_STREAM_GLOBAL_BLOCKING) {
        g_counters.host_syncs++;
        APCG_HIP(hipStreamSynchronize(c->stream));
    }
    return APCG_SUCCESS;
}

apcg_status ensure_workspace(apcg_ctx c, int64_t n) {
    if (n < 1) n = 1;
    if (c->ws.base && c->ws.cap >= n) return APCG_SUCCESS;
    // the old workspace may still be in use by queued work on this stream
    if (c->ws.base) {
        EventRef ev = event_get(c->device);
        if (!ev) return set_error(APCG_ERR_HIP, "event creation failed");
        APCG_HIP(hipEventRecord(ev->e, c->stream));
        double *old = c->ws.base;
        int dev = c->device;
        // graphs captured with the old buffers are stale now
        std::vector<GraphEntry> gs;
        gs.swap(c->graphs);
        defer_release({ev}, [old, dev, gs]() {
            hipSetDevice(dev);
            for (auto &g : gs) {
                if (g.exec) hipGraphExecDestroy(g.exec);
                if (g.graph) hipGraphDestroy(g.graph);
            }
            hipFree(old);
        });
        c->ws.base = nullptr;
    }
    int64_t cap = ((n + 63) / 64) * 64;
    APCG_HIP(hipMalloc((void **)&c->ws.base, sizeof(double) * 6 * cap));
    c->ws.cap = cap;
    if (!c->ws.state) APCG_HIP(hipMalloc((void **)&c->ws.state, 256));
    return APCG_SUCCESS;
}

int32_t normalise_blocks(int32_t blocks, int64_t units) {
    int64_t b = blocks > 0 ? blocks : 2048;
    if (units < 1) units = 1;
    if (b > units) b = units;
    b = ((b + 7) / 8) * 8;
    if (b > kMaxBlocks) b = kMaxBlocks;
    if (b < 8) b = 8;
    return (int32_t)b;
}

void spmv_default_config(int32_t n, int64_t nnz, apcg_spmv_config *cfg) {
    double per_row = n > 0 ? (double)nnz / n : 0.0;
    int lpr = 1;
    while (lpr < 64 && lpr * 4 <= per_row) lpr *= 2;  // about four entries per lane
    cfg->lanes_per_row = lpr;
    cfg->block_size = 256;
    cfg->blocks = 1024;
    cfg->schedule = APCG_SPMV_ROWGROUP;
}

}  // namespace apcg

using namespace apcg;

#define API_BEGIN() \
    try {
#define API_END()                                                        \
    }                                                                    \
    catch (const std::bad_alloc &) {                                     \
        return set_error(APCG_ERR_OUT_OF_MEMORY, "host allocation failed"); \
    }                                                                    \
    catch (...) {                                                        \
        return set_error(APCG_ERR_INVALID_STATE, "unexpected exception"); \
    }

static apcg_status check_device(int32_t device) {
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || count <= 0)
        return set_error(APCG_ERR_UNSUPPORTED, "no HIP device available");
    if (device < 0 || device >= count) return set_error(APCG_ERR_INVALID_ARG, "device index out of range");
    return APCG_SUCCESS;
}

extern "C" {

int32_t apcg_abi_version(void) { return APCG_ABI_VERSION; }

const char *apcg_last_error(void) { return t_last_error.c_str(); }

apcg_status apcg_device_count(int32_t *count) {
    if (!count) return set_error(APCG_ERR_INVALID_ARG, "count is NULL");
    int c = 0;
    if (hipGetDeviceCount(&c) != hipSuccess) c = 0;
    *count = c;
    return APCG_SUCCESS;
}

apcg_status apcg_device_props_get(int32_t device, apcg_device_props *out) {
    API_BEGIN();
    if (!out) return set_error(APCG_ERR_INVALID_ARG, "out is NULL");
    apcg_status s = check_device(device);
    if (s) return s;
    hipDeviceProp_t p;
    APCG_HIP(hipGetDeviceProperties(&p, device));
    memset(out, 0, sizeof *out);
    snprintf(out->name, sizeof out->name, "%s", p.name);
    snprintf(out->arch, sizeof out->arch, "%s", p.gcnArchName);
    out->compute_units = p.multiProcessorCount;
    out->wavefront_size = p.warpSize;
    out->global_mem_bytes = (int64_t)p.totalGlobalMem;
    out->clock_khz = p.clockRate;
    out->l2_bytes = p.l2CacheSize;
    out->lds_bytes_per_block = (int32_t)p.sharedMemPerBlock;
    return APCG_SUCCESS;
    API_END();
}

// ----------------------------------------------------------------- contexts

apcg_status apcg_ctx_create(int32_t device, int32_t stream_type, apcg_ctx *out) {
    API_BEGIN();
    if (!out) return set_error(APCG_ERR_INVALID_ARG, "out is NULL");
    if (stream_type != APCG_STREAM_DEFAULT && stream_type != APCG_STREAM_GLOBAL_BLOCKING)
        return set_error(APCG_ERR_INVALID_ARG, "unknown stream type");
    apcg_status s = check_device(device);
    if (s) return s;
    reap();
    apcg_ctx c = new apcg_ctx_s();
    s = ctx_init(c, device, stream_type);
    if (s) {
        ctx_release_now(c);
        return s;
    }
    *out = c;
    return APCG_SUCCESS;
    API_END();
}

apcg_status apcg_ctx_destroy(apcg_ctx ctx) {
    API_BEGIN();
    if (!ctx) return set_error(APCG_ERR_INVALID_ARG, "ctx is NULL");
    if (ctx->is_default_global) return set_error(APCG_ERR_INVALID_ARG, "the default context cannot be destroyed");
    APCG_HIP(hipSetDevice(ctx->device));
    EventRef ev = event_get(ctx->device);
    if (!ev) return set_error(APCG_ERR_HIP, "event creation failed");
    APCG_HIP(hipEventRecord(ev->e, ctx->stream));
    defer_release({ev}, [ctx]() { ctx_release_now(ctx); });
    reap();
    return APCG_SUCCESS;
    API_END();
}

apcg_status apcg_ctx_wait_for(apcg_ctx waiter, apcg_ctx waitee) {
    API_BEGIN();
    if (!waiter || !waitee) return set_error(APCG_ERR_INVALID_ARG, "NULL context");
    if (waiter == waitee) return APCG_SUCCESS;
    APCG_HIP(hipSetDevice(waitee->device));
    EventRef ev = event_get(waitee->device);
    if (!ev) return set_error(APCG_ERR_HIP, "event creation failed");
    APCG_HIP(hipEventRecord(ev->e, waitee->stream));
    APCG_HIP(hipSetDevice(waiter->device));
    g_counters.stream_waits++;
    APCG_HIP(hipStreamWaitEvent(waiter->stream, ev->e, 0));
    return APCG_SUCCESS;
    API_END();
}

apcg_status apcg_ctx_query_idle(apcg_ctx ctx, int32_t *idle) {
    API_BEGIN();
    if (!ctx || !idle) return set_error(APCG_ERR_INVALID_ARG, "NULL argument");
    APCG_HIP(hipSetDevice(ctx->device));
    hipError_t e = hipStreamQuery(ctx->stream);
    if (e == hipSuccess) *idle = 1;
    else if (e == hipErrorNotReady) *idle = 0;
    else return hip_error(e, "hipStreamQuery");
    return APCG_SUCCESS;
    API_END();
}

apcg_status apcg_ctx_synchronize(apcg_ctx ctx) {
    API_BEGIN();
    if (!ctx) return set_error(APCG_ERR_INVALID_ARG, "ctx is NULL");
    APCG_HIP(hipSetDevice(ctx->device));
    g_counters.host_syncs++;
    APCG_HIP(hipStreamSynchronize(ctx->stream));
    reap();
    return APCG_SUCCESS;
    API_END();
}

apcg_status apcg_ctx_get_stream_type(apcg_ctx ctx, int32_t *stream_type) {
    if (!ctx || !stream_type) return set_error(APCG_ERR_INVALID_ARG, "NULL argument");
    *stream_type = ctx->type;
    return APCG_SUCCESS;
}

apcg_status apcg_ctx_fork(apcg_ctx parent, int32_t n, apcg_ctx *children) {
    API_BEGIN();
    if (!parent || (n > 0 && !children) || n < 0) return set_error(APCG_ERR_INVALID_ARG, "bad fork arguments");
    APCG_HIP(hipSetDevice(parent->device));
    EventRef ev = event_get(parent->device);
    if (!ev) return set_error(APCG_ERR_HIP, "event creation failed");
    APCG_HIP(hipEventRecord(ev->e, parent->stream));
    for (int32_t i = 0; i < n; ++i) {
        apcg_ctx c = new apcg_ctx_s();
        apcg_status s = ctx_init(c, parent->device, parent->type == APCG_STREAM_GLOBAL_BLOCKING
                                                        ? APCG_STREAM_GLOBAL_BLOCKING
                                                        : APCG_STREAM_DEFAULT);
        if (s) {
            ctx_release_now(c);
            for (int32_t j = 0; j < i; ++j) apcg_ctx_destroy(children[j]);
            return s;
        }
        g_counters.stream_waits++;
        APCG_HIP(hipStreamWaitEvent(c->stream, ev->e, 0));
        children[i] = c;
    }
    return APCG_SUCCESS;
    API_END();
}

apcg_status apcg_ctx_join(apcg_ctx parent, int32_t n, int32_t mode, apcg_ctx *children) {
    API_BEGIN();
    if (!parent || n < 0 || (n > 0 && !children)) return set_error(APCG_ERR_INVALID_ARG, "bad join arguments");
    if (mode != APCG_JOIN_DESTROY && mode != APCG_JOIN_SYNC && mode != APCG_JOIN_NO_SYNC)
        return set_error(APCG_ERR_INVALID_ARG, "unknown join mode");
    for (int32_t i = 0; i < n; ++i)
        if (!children[i] || children[i] == parent) return set_error(APCG_ERR_INVALID_ARG, "bad child context");
    for (int32_t i = 0; i < n; ++i) {
        apcg_status s = apcg_ctx_wait_for(parent, children[i]);
        if (s) return s;
    }
    for (int32_t i = 0; i < n; ++i) {
        if (mode == APCG_JOIN_SYNC) {
            apcg_status s = apcg_ctx_synchronize(children[i]);
            if (s) return s;
        } else if (mode == APCG_JOIN_DESTROY) {
            apcg_status s = apcg_ctx_destroy(children[i]);
            if (s) return s;
            children[i] = nullptr;
        }
    }
    return APCG_SUCCESS;
    API_END();
}

// ----------------------------------------------------------------- scalars

static std::mutex g_scalar_mu;
struct ScalarPool {
    std::vector<double *> chunks;
    std::vector<int64_t> free_slots;
};
static std::map<int, ScalarPool> g_scalar_pool;
constexpr int64_t kScalarChunk = 4096;

static apcg_status scalar_slot_alloc(int device, double **ptr, int64_t *slot) {
    std::lock_guard<std::mutex> lk(g_scalar_mu);
    ScalarPool &p = g_scalar_pool[device];
    if (p.free_slots.empty()) {
        double *chunk = nullptr;
        APCG_HIP(hipSetDevice(device));
        APCG_HIP(hipMalloc((void **)&chunk, sizeof(double) * kScalarChunk));
        int64_t base = (int64_t)p.chunks.size() * kScalarChunk;
        p.chunks.push_back(chunk);
        for (int64_t i = kScalarChunk - 1; i >= 0; --i) p.free_slots.push_back(base + i);
    }
    int64_t s = p.free_slots.back();
    p.free_slots.pop_back();
    *slot = s;
    *ptr = p.chunks[s / kScalarChunk] + (s % kScalarChunk);
    return APCG_SUCCESS;
}

static void scalar_slot_free(int device, int64_t slot) {
    std::lock_guard<std::mutex> lk(g_scalar_mu);
    g_scalar_pool[device].free_slots.push_back(slot);
}

apcg_status apcg_scalar_create(apcg_ctx ctx, apcg_scalar *out) {
    API_BEGIN();
    if (!out) return set_error(APCG_ERR_INVALID_ARG, "out is NULL");
    int device = 0;
    if (ctx) device = ctx->device;
    else {
        apcg_status s0 = check_device(0);
        if (s0) return s0;
    }
    apcg_ctx c = nullptr;
    apcg_status s = resolve_ctx(ctx, device, &c);
    if (s) return s;
    apcg_scalar sc = new apcg_scalar_s();
    sc->device = device;
    s = scalar_slot_alloc(device, &sc->d, &sc->slot);
    if (s) {
        delete sc;
        return s;
    }
    Acc acc[1] = {{&sc->rec, ACC_W}};
    if ((s = op_begin(c, acc, 1))) return s;
    if ((s = launch_scalar_set(c->stream, sc->d, 0.0))) return s;
    if ((s = op_end(c, acc, 1))) return s;
    *out = sc;
    return APCG_SUCCESS;
    API_END();
}

apcg_status apcg_scalar_destroy(apcg_scalar s) {
    API_BEGIN();
    if (!s) return set_error(APCG_ERR_INVALID_ARG, "scalar is NULL");
    std::vector<EventRef> deps;
    {
        std::lock_guard<std::recursive_mutex> lk(g_mu);
        deps = record_deps(s->rec);
    }
    int dev = s->device;
    int64_t slot = s->slot;
    if (s->mark_id) intent_forget(s->mark_id);
    delete s;
    defer_release(std::move(deps), [dev, slot]() { scalar_slot_free(dev, slot); });
    reap();
    return APCG_SUCCESS;
    API_END();
}

apcg_status apcg_scalar_set(apcg_scalar sc, double value, apcg_ctx ctx) {
    API_BEGIN();
    if (!sc) return set_error(APCG_ERR_INVALID_ARG, "scalar is NULL");
    apcg_ctx c = nullptr;
    apcg_status s = resolve_ctx(ctx, sc->device, &c);
    if (s) return s;
    Acc acc[1] = {{&sc->rec, ACC_W}};
    if ((s = op_begin(c, acc, 1))) return s;
    if ((s = launch_scalar_set(c->stream, sc->d, value))) return s;
    return op_end(c, acc, 1);
    API_END();
}

static apcg_status wait_last_writer(const Record &r, int device) {
    EventRef ev;
    {
        std::lock_guard<std::recursive_mutex> lk(g_mu);
        ev = r.write_ev;
    }
    APCG_HIP(hipSetDevice(device));
    if (ev && ev->e) {
        g_counters.host_syncs++;
        APCG_HIP(hipEventSynchronize(ev->e));
    }
    return APCG_SUCCESS;
}

apcg_status apcg_scalar_get(apcg_scalar sc, double *host_value) {
    API_BEGIN();
    if (!sc || !host_value) return set_error(APCG_ERR_INVALID_ARG, "NULL argument");
    apcg_status s = wait_last_writer(sc->rec, sc->device);
    if (s) return s;
    g_counters.d2h_copies++;
    APCG_HIP(hipMemcpy(host_value, sc->d, sizeof(double), hipMemcpyDeviceToHost));
    reap();
    return APCG_SUCCESS;
    API_END();
}

apcg_status apcg_scalar_op(int32_t opcode, apcg_scalar out, apcg_scalar a, apcg_scalar b, apcg_ctx ctx) {
    API_BEGIN();
    if (!out || !a) return set_error(APCG_ERR_INVALID_ARG, "NULL scalar");
    bool binary = opcode >= APCG_SCALAR_ADD && opcode <= APCG_SCALAR_DIV;
    bool unary = opcode >= APCG_SCALAR_COPY && opcode <= APCG_SCALAR_SQRT;
    if (!binary && !unary) return set_error(APCG_ERR_INVALID_ARG, "unknown scalar opcode");
    if (binary && !b) return set_error(APCG_ERR_INVALID_ARG, "binary opcode needs b");
    if (unary && b) return set_error(APCG_ERR_INVALID_ARG, "unary opcode takes no b");
    if (a->device != out->device || (b && b->device != out->device))
        return set_error(APCG_ERR_INVALID_ARG, "scalars on different devices");
    apcg_ctx c = nullptr;
    apcg_status s = resolve_ctx(ctx, out->device, &c);
    if (s) return s;
    Acc acc[3];
    int na = 0;
    acc[na++] = {&out->rec, ACC_W};
    if (a != out) acc[na++] = {&a->rec, ACC_R};
    if (b && b != out && b != a) acc[na++] = {&b->rec, ACC_R};
    if ((s = op_begin(c, acc, na))) return s;
    if ((s = launch_scalar_op(c->stream, opcode, out->d, a->d, b ? b->d : nullptr))) return s;
    return op_end(c, acc, na);
    API_END();
}

// ----------------------------------------------------------------- vectors

apcg_status apcg_vec_wrap(int32_t device, double *dev_ptr, int64_t n, apcg_vec *out) {
    API_BEGIN();
    if (!out || n < 0 || (n > 0 && !dev_ptr)) return set_error(APCG_ERR_INVALID_ARG, "bad vector arguments");
    if (((uintptr_t)dev_ptr) % 8 != 0) return set_error(APCG_ERR_INVALID_ARG, "vector pointer not 8-byte aligned");
    apcg_status s = check_device(device);
    if (s) return s;
    apcg_vec v = new apcg_vec_s();
    v->device = device;
    v->d = dev_ptr;
    v->n = n;
    *out = v;
    return APCG_SUCCESS;
    API_END();
}

apcg_status apcg_vec_destroy(apcg_vec v) {
    API_BEGIN();
    if (!v) return set_error(APCG_ERR_INVALID_ARG, "vector is NULL");
    std::vector<EventRef> deps;
    {
        std::lock_guard<std::recursive_mutex> lk(g_mu);
        deps = record_deps(v->rec);
    }
    if (v->mark_id) intent_forget(v->mark_id);
    delete v;
    defer_release(std::move(deps), []() {});
    reap();
    return APCG_SUCCESS;
    API_END();
}

static apcg_status vec_ctx(apcg_vec v, apcg_ctx ctx, apcg_ctx *c) {
    if (!v) return set_error(APCG_ERR_INVALID_ARG, "vector is NULL");
    return resolve_ctx(ctx, v->device, c);
}

apcg_status apcg_vec_dot_async(apcg_vec x, apcg_vec y, apcg_scalar out, apcg_ctx ctx) {
    API_BEGIN();
    if (!x || !y || !out) return set_error(APCG_ERR_INVALID_ARG, "NULL argument");
    if (x->n != y->n) return set_error(APCG_ERR_INVALID_ARG, "vector lengths differ");
    if (x->device != y->device || out->device != x->device)
        return set_error(APCG_ERR_INVALID_ARG, "operands on different devices");
    apcg_ctx c = nullptr;
    apcg_status s = vec_ctx(x, ctx, &c);
    if (s) return s;
    Acc acc[3] = {{&out->rec, ACC_W}, {&x->rec, ACC_R}, {&y->rec, ACC_R}};
    int na = (x == y) ? 2 : 3;
    if ((s = op_begin(c, acc, na))) return s;
    if ((s = launch_dot(c->stream, x->d, y->d, x->n, out->d, 0, c->partials))) return s;
    return op_end(c, acc, na);
    API_END();
}

apcg_status apcg_vec_norm2_async(apcg_vec x, apcg_scalar out, apcg_ctx ctx) {
    API_BEGIN();
    if (!x || !out) return set_error(APCG_ERR_INVALID_ARG, "NULL argument");
    if (out->device != x->device) return set_error(APCG_ERR_INVALID_ARG, "operands on different devices");
    apcg_ctx c = nullptr;
    apcg_status s = vec_ctx(x, ctx, &c);
    if (s) return s;
    Acc acc[2] = {{&out->rec, ACC_W}, {&x->rec, ACC_R}};
    if ((s = op_begin(c, acc, 2))) return s;
    if ((s = launch_dot(c->stream, x->d, x->d, x->n, out->d, 1, c->partials))) return s;
    return op_end(c, acc, 2);
    API_END();
}

apcg_status apcg_vec_axpy_async(apcg_vec y, apcg_scalar a, int32_t negate, apcg_vec x, apcg_ctx ctx) {
    API_BEGIN();
    if (!x || !y || !a) return set_error(APCG_ERR_INVALID_ARG, "NULL argument");
    if (x->n != y->n) return set_error(APCG_ERR_INVALID_ARG, "vector lengths differ");
    if (x->device != y->device || a->device != y->device)
        return set_error(APCG_ERR_INVALID_ARG, "operands on different devices");
    apcg_ctx c = nullptr;
    apcg_status s = vec_ctx(y, ctx, &c);
    if (s) return s;
    Acc acc[3] = {{&y->rec, ACC_RW}, {&a->rec, ACC_R}, {&x->rec, ACC_R}};
    int na = (x == y) ? 2 : 3;
    if ((s = op_begin(c, acc, na))) return s;
    if ((s = launch_axpy(c->stream, y->d, a->d, negate ? -1.0 : 1.0, x->d, y->n))) return s;
    return op_end(c, acc, na);
    API_END();
}

apcg_status apcg_vec_aypx_async(apcg_vec y, apcg_scalar b, apcg_vec x, apcg_ctx ctx) {
    API_BEGIN();
    if (!x || !y || !b) return set_error(APCG_ERR_INVALID_ARG, "NULL argument");
    if (x->n != y->n) return set_error(APCG_ERR_INVALID_ARG, "vector lengths differ");
    if (x->device != y->device || b->device != y->device)
        return set_error(APCG_ERR_INVALID_ARG, "operands on different devices");
    apcg_ctx c = nullptr;
    apcg_status s = vec_ctx(y, ctx, &c);
    if (s) return s;
    Acc acc[3] = {{&y->rec, ACC_RW}, {&b->rec, ACC_R}, {&x->rec, ACC_R}};
    int na = (x == y) ? 2 : 3;
    if ((s = op_begin(c, acc, na))) return s;
    if ((s = launch_aypx(c->stream, y->d, b->d, x->d, y->n))) return s;
    return op_end(c, acc, na);
    API_END();
}

apcg_status apcg_vec_scale_async(apcg_vec x, apcg_scalar a, apcg_ctx ctx) {
    API_BEGIN();
    if (!x || !a) return set_error(APCG_ERR_INVALID_ARG, "NULL argument");
    if (a->device != x->device) return set_error(APCG_ERR_INVALID_ARG, "operands on different devices");
    apcg_ctx c = nullptr;
    apcg_status s = vec_ctx(x, ctx, &c);
    if (s) return s;
    Acc acc[2] = {{&x->rec, ACC_RW}, {&a->rec, ACC_R}};
    if ((s = op_begin(c, acc, 2))) return s;
    if ((s = launch_scale(c->stream, x->d, a->d, x->n))) return s;
    return op_end(c, acc, 2);
    API_END();
}

apcg_status apcg_vec_copy_async(apcg_vec dst, apcg_vec src, apcg_ctx ctx) {
    API_BEGIN();
    if (!dst || !src) return set_error(APCG_ERR_INVALID_ARG, "NULL argument");
    if (dst->n != src->n) return set_error(APCG_ERR_INVALID_ARG, "vector lengths differ");
    if (dst->device != src->device) return set_error(APCG_ERR_INVALID_ARG, "operands on different devices");
    if (dst == src) return APCG_SUCCESS;
    apcg_ctx c = nullptr;
    apcg_status s = vec_ctx(dst, ctx, &c);
    if (s) return s;
    Acc acc[2] = {{&dst->rec, ACC_W}, {&src->rec, ACC_R}};
    if ((s = op_begin(c, acc, 2))) return s;
    if ((s = launch_copy(c->stream, dst->d, src->d, dst->n))) return s;
    return op_end(c, acc, 2);
    API_END();
}

apcg_status apcg_vec_set_async(apcg_vec x, double value, apcg_ctx ctx) {
    API_BEGIN();
    apcg_ctx c = nullptr;
    apcg_status s = vec_ctx(x, ctx, &c);
    if (s) return s;
    Acc acc[1] = {{&x->rec, ACC_W}};
    if ((s = op_begin(c, acc, 1))) return s;
    if ((s = launch_fill(c->stream, x->d, value, x->n))) return s;
    return op_end(c, acc, 1);
    API_END();
}

apcg_status apcg_vec_copy_to_host(apcg_vec x, double *host_out) {
    API_BEGIN();
    if (!x || (x->n > 0 && !host_out)) return set_error(APCG_ERR_INVALID_ARG, "NULL argument");
    apcg_status s = wait_last_writer(x->rec, x->device);
    if (s) return s;
    if (x->n > 0) {
        g_counters.d2h_copies++;
        APCG_HIP(hipMemcpy(host_out, x->d, sizeof(double) * x->n, hipMemcpyDeviceToHost));
    }
    reap();
    return APCG_SUCCESS;
    API_END();
}

apcg_status apcg_vec_copy_from_host(apcg_vec x, const double *host_in, apcg_ctx ctx) {
    API_BEGIN();
    if (!x || (x->n > 0 && !host_in)) return set_error(APCG_ERR_INVALID_ARG, "NULL argument");
    apcg_ctx c = nullptr;
    apcg_status s = vec_ctx(x, ctx, &c);
    if (s) return s;
    Acc acc[1] = {{&x->rec, ACC_W}};
    if ((s = op_begin(c, acc, 1))) return s;
    if (x->n > 0) {
        g_counters.h2d_copies++;
        APCG_HIP(hipMemcpyAsync(x->d, host_in, sizeof(double) * x->n, hipMemcpyHostToDevice, c->stream));
        // the host buffer may be reused as soon as the call returns
        g_counters.host_syncs++;
        APCG_HIP(hipStreamSynchronize(c->stream));
    }
    return op_end(c, acc, 1);
    API_END();
}

// ----------------------------------------------------------------- matrices

apcg_status apcg_mat_wrap_csr(int32_t device, int32_t n, int64_t nnz, const int32_t *dev_rowptr,
                              const int32_t *dev_col, const double *dev_val, const int32_t *host_rowptr,
                              apcg_mat *out) {
    API_BEGIN();
    if (!out || n < 0 || nnz < 0 || !dev_rowptr || (nnz > 0 && (!dev_col || !dev_val)))
        return set_error(APCG_ERR_INVALID_ARG, "bad CSR arguments");
    if (nnz > INT32_MAX) return set_error(APCG_ERR_UNSUPPORTED, "nnz exceeds the int32 index range");
    apcg_status s = check_device(device);
    if (s) return s;
    std::vector<int32_t> tmp;
    const int32_t *rp = host_rowptr;
    if (!rp) {
        tmp.resize((size_t)n + 1);
        APCG_HIP(hipSetDevice(device));
        g_counters.d2h_copies++;
        APCG_HIP(hipMemcpy(tmp.data(), dev_rowptr, sizeof(int32_t) * ((size_t)n + 1), hipMemcpyDeviceToHost));
        rp = tmp.data();
    }
    if (rp[0] != 0 || rp[n] != (int32_t)nnz) return set_error(APCG_ERR_INVALID_ARG, "rowptr[0] != 0 or rowptr[n] != nnz");
    for (int32_t i = 0; i < n; ++i)
        if (rp[i + 1] < rp[i]) return set_error(APCG_ERR_INVALID_ARG, "rowptr is decreasing");
    apcg_mat A = new apcg_mat_s();
    A->uid = g_next_id++;
    A->device = device;
    A->n = n;
    A->nnz = nnz;
    A->rowptr = dev_rowptr;
    A->col = dev_col;
    A->val = dev_val;
    for (int t = 0; t < 2; ++t) {
        const int64_t rows = t == 0 ? 256 : 512;
        int64_t mx = 0;
        for (int64_t r0 = 0; r0 < n; r0 += rows) mx = std::max<int64_t>(mx, rp[std::min<int64_t>(n, r0 + rows)] - rp[r0]);
        A->max_block_nnz[t] = mx;
    }
    {  // 64-row slices: offset and width (longest row) of each
        const int64_t nsl = ((int64_t)n + 63) / 64;
        A->sell_meta_h.resize(2 * nsl);
        int64_t off = 0;
        int32_t maxw = 0;
        for (int64_t sl = 0; sl < nsl; ++sl) {
            int32_t w = 0;
            for (int64_t i = sl * 64; i < std::min<int64_t>(n, sl * 64 + 64); ++i) w = std::max(w, rp[i + 1] - rp[i]);
            A->sell_meta_h[2 * sl] = (int32_t)std::min<int64_t>(off, INT32_MAX);
            A->sell_meta_h[2 * sl + 1] = w;
            off += 64 * (int64_t)w;
            maxw = std::max(maxw, w);
        }
        A->sell_entries = off > INT32_MAX ? -1 : off;
        A->sell_maxw = maxw;
    }
    spmv_default_config(n, nnz, &A->cfg);
    if (stream_fits(A, 256)) A->cfg = apcg_spmv_config{1, 256, 1024, APCG_SPMV_STREAM};
    *out = A;
    return APCG_SUCCESS;
    API_END();
}

apcg_status apcg_mat_destroy(apcg_mat A) {
    API_BEGIN();
    if (!A) return set_error(APCG_ERR_INVALID_ARG, "matrix is NULL");
    std::vector<EventRef> deps;
    {
        std::lock_guard<std::recursive_mutex> lk(g_mu);
        deps = record_deps(A->rec);
    }
    const int dev = A->device;
    int32_t *smeta = A->sell_meta, *scol = A->sell_col, *doff = A->sdia_off, *gtab = A->dia_tab;
    double *sval = A->sell_val, *dval = A->sdia_val, *gval = A->dia_val;
    uint64_t *dmsk = A->sdia_msk;
    if (A->mark_id) intent_forget(A->mark_id);
    delete A;
    defer_release(std::move(deps), [dev, smeta, scol, sval, doff, dmsk, dval, gtab, gval]() {
        if (smeta || scol || sval || doff || dmsk || dval || gtab || gval) {
            hipSetDevice(dev);
            hipFree(smeta);
            hipFree(scol);
            hipFree(sval);
            hipFree(doff);
            hipFree(dmsk);
            hipFree(dval);
            hipFree(gtab);
            hipFree(gval);
        }
    });
    reap();
    return APCG_SUCCESS;
    API_END();
}

static bool valid_spmv_config(const apcg_spmv_config *cfg) {
    int l = cfg->lanes_per_row, b = cfg->block_size;
    bool lok = l == 1 || l == 2 || l == 4 || l == 8 || l == 16 || l == 32 || l == 64;
    if (cfg->schedule == APCG_SPMV_SDIA) lok = l >= 1 && l <= 64;  // planes per marching task
    if (cfg->schedule == APCG_SPMV_DIA) lok = l >= 1 && l <= 64;  // > 1: planes per marching task
    bool bok = b == 256 || b == 512;
    bool sok = cfg->schedule == APCG_SPMV_ROWGROUP || cfg->schedule == APCG_SPMV_STREAM ||
               cfg->schedule == APCG_SPMV_SELL || cfg->schedule == APCG_SPMV_SDIA || cfg->schedule == APCG_SPMV_DIA;
    return lok && bok && sok && cfg->blocks >= 0;
}

apcg_status apcg_mat_set_spmv_config(apcg_mat A, const apcg_spmv_config *cfg) {
    if (!A || !cfg) return set_error(APCG_ERR_INVALID_ARG, "NULL argument");
    if (!valid_spmv_config(cfg))
        return set_error(APCG_ERR_INVALID_ARG, "invalid SpMV configuration (block_size must be 256 or 512)");
    if (cfg->schedule == APCG_SPMV_STREAM && !stream_fits(A, cfg->block_size))
        return set_error(APCG_ERR_UNSUPPORTED, "rows too long for the staged schedule at this block size");
    if (cfg->schedule == APCG_SPMV_SELL && A->sell_entries < 0)
        return set_error(APCG_ERR_UNSUPPORTED, "matrix too large for the sliced layout's int32 offsets");
    if (cfg->schedule == APCG_SPMV_SDIA) {
        apcg_status s = apcg::sdia_analyse(A);
        if (s) return s;
        if (A->sdia_state < 0) return set_error(APCG_ERR_UNSUPPORTED, A->sdia_reason);
    }
    if (cfg->schedule == APCG_SPMV_DIA) {
        apcg_status s = apcg::dia_analyse(A);
        if (s) return s;
        if (A->dia_state < 0) return set_error(APCG_ERR_UNSUPPORTED, A->dia_reason);
    }
    A->cfg = *cfg;
    return APCG_SUCCESS;
}

apcg_status apcg_mat_get_sdia_info(apcg_mat A, int32_t out[6]) {
    if (!A || !out) return set_error(APCG_ERR_INVALID_ARG, "NULL argument");
    out[0] = A->sdia_state;
    out[1] = A->sdia_u;
    out[2] = A->sdia_mp;
    out[3] = A->sdia_ps;
    out[4] = A->sdia_sym;
    out[5] = 0;
    if (A->sdia_state == 1 && A->sdia_off) {
        // the flag word after the offsets and the partner slots; every queued
        // refill and check has finished once the device is idle
        const int64_t nsl = ((int64_t)A->n + 63) / 64;
        APCG_HIP(hipSetDevice(A->device));
        apcg::g_counters.host_syncs++;
        APCG_HIP(hipDeviceSynchronize());
        apcg::g_counters.d2h_copies++;
        APCG_HIP(hipMemcpy(&out[5], A->sdia_off + 2 * nsl * A->sdia_mp, sizeof(int32_t), hipMemcpyDeviceToHost));
    }
    return APCG_SUCCESS;
}

apcg_status apcg_mat_get_dia_info(apcg_mat A, int32_t out[4]) {
    if (!A || !out) return set_error(APCG_ERR_INVALID_ARG, "NULL argument");
    out[0] = A->dia_state;
    out[1] = A->dia_nd;
    out[2] = A->dia_sym;
    out[3] = 0;
    if (A->dia_state == 1 && A->dia_tab) {
        APCG_HIP(hipSetDevice(A->device));
        apcg::g_counters.host_syncs++;
        APCG_HIP(hipDeviceSynchronize());
        apcg::g_counters.d2h_copies++;
        APCG_HIP(hipMemcpy(&out[3], A->dia_tab + 18, sizeof(int32_t), hipMemcpyDeviceToHost));
    }
    return APCG_SUCCESS;
}

apcg_status apcg_mat_get_spmv_config(apcg_mat A, apcg_spmv_config *cfg) {
    if (!A || !cfg) return set_error(APCG_ERR_INVALID_ARG, "NULL argument");
    *cfg = A->cfg;
    return APCG_SUCCESS;
}

apcg_status apcg_mat_mult_async(apcg_mat A, apcg_vec x, apcg_vec y, apcg_ctx ctx) {
    API_BEGIN();
    if (!A || !x || !y) return set_error(APCG_ERR_INVALID_ARG, "NULL argument");
    if (x->n != A->n || y->n != A->n) return set_error(APCG_ERR_INVALID_ARG, "dimension mismatch");
    if (vec_overlap(x, y)) return set_error(APCG_ERR_INVALID_ARG, "x and y must not share memory");
    if (x->device != A->device || y->device != A->device)
        return set_error(APCG_ERR_INVALID_ARG, "operands on different devices");
    apcg_ctx c = nullptr;
    apcg_status s = resolve_ctx(ctx, A->device, &c);
    if (s) return s;
    Acc acc[3] = {{&y->rec, ACC_W}, {&A->rec, ACC_R}, {&x->rec, ACC_R}};
    if ((s = op_begin(c, acc, 3))) return s;
    if ((s = launch_spmv(c->stream, A, x->d, y->d))) return s;
    return op_end(c, acc, 3);
    API_END();
}

// ----------------------------------------------------------------- info

apcg_status apcg_info_create(int32_t device, int32_t count, apcg_info *out) {
    API_BEGIN();
    if (!out || count < 1) return set_error(APCG_ERR_INVALID_ARG, "bad info arguments");
    apcg_status s = check_device(device);
    if (s) return s;
    apcg_info in = new apcg_info_s();
    in->device = device;
    in->count = count;
    APCG_HIP(hipSetDevice(device));
    hipError_t e = hipMalloc((void **)&in->d, sizeof(apcg_solve_info) * count);
    if (e != hipSuccess) {
        delete in;
        return hip_error(e, "hipMalloc(info)");
    }
    APCG_HIP(hipMemset(in->d, 0, sizeof(apcg_solve_info) * count));
    *out = in;
    return APCG_SUCCESS;
    API_END();
}

apcg_status apcg_info_destroy(apcg_info info) {
    API_BEGIN();
    if (!info) return set_error(APCG_ERR_INVALID_ARG, "info is NULL");
    std::vector<EventRef> deps;
    {
        std::lock_guard<std::recursive_mutex> lk(g_mu);
        deps = record_deps(info->rec);
    }
    apcg_solve_info *d = info->d;
    int dev = info->device;
    delete info;
    defer_release(std::move(deps), [d, dev]() {
        hipSetDevice(dev);
        hipFree(d);
    });
    reap();
    return APCG_SUCCESS;
    API_END();
}

apcg_status apcg_info_get(apcg_info info, int32_t index, apcg_solve_info *out) {
    API_BEGIN();
    if (!info || !out) return set_error(APCG_ERR_INVALID_ARG, "NULL argument");
    if (index < 0 || index >= info->count) return set_error(APCG_ERR_INVALID_ARG, "info index out of range");
    apcg_status s = wait_last_writer(info->rec, info->device);
    if (s) return s;
    g_counters.d2h_copies++;
    APCG_HIP(hipMemcpy(out, info->d + index, sizeof(apcg_solve_info), hipMemcpyDeviceToHost));
    reap();
    return APCG_SUCCESS;
    API_END();
}

// ----------------------------------------------------------------- timers

apcg_status apcg_timer_create(apcg_timer *out) {
    if (!out) return set_error(APCG_ERR_INVALID_ARG, "out is NULL");
    *out = new apcg_timer_s();
    return APCG_SUCCESS;
}

apcg_status apcg_timer_destroy(apcg_timer t) {
    if (!t) return set_error(APCG_ERR_INVALID_ARG, "timer is NULL");
    std::vector<EventRef> deps;
    if (t->start) deps.push_back(t->start);
    if (t->stop) deps.push_back(t->stop);
    EventRef a = t->start, b = t->stop;
    delete t;
    // timing events are destroyed, not pooled, once they have completed
    defer_release(deps, [a, b]() mutable {
        for (EventRef *e : {&a, &b})
            if (*e && (*e)->e) {
                hipEventDestroy((*e)->e);
                (*e)->e = nullptr;
            }
    });
    reap();
    return APCG_SUCCESS;
}

static apcg_status timer_mark(EventRef *slot, apcg_ctx ctx) {
    if (!ctx) return set_error(APCG_ERR_INVALID_ARG, "ctx is NULL");
    APCG_HIP(hipSetDevice(ctx->device));
    if (!*slot || (*slot)->device != -1 - ctx->device) {
        *slot = timing_event_get(ctx->device);
        if (!*slot) return set_error(APCG_ERR_HIP, "event creation failed");
    }
    APCG_HIP(hipEventRecord((*slot)->e, ctx->stream));
    return APCG_SUCCESS;
}

apcg_status apcg_timer_start(apcg_timer t, apcg_ctx ctx) {
    if (!t) return set_error(APCG_ERR_INVALID_ARG, "timer is NULL");
    return timer_mark(&t->start, ctx);
}

apcg_status apcg_timer_stop(apcg_timer t, apcg_ctx ctx) {
    if (!t) return set_error(APCG_ERR_INVALID_ARG, "timer is NULL");
    return timer_mark(&t->stop, ctx);
}

apcg_status apcg_timer_elapsed_ms(apcg_timer t, double *ms) {
    if (!t || !ms) return set_error(APCG_ERR_INVALID_ARG, "NULL argument");
    if (!t->start || !t->stop) return set_error(APCG_ERR_INVALID_STATE, "timer not started and stopped");
    g_counters.host_syncs++;
    APCG_HIP(hipEventSynchronize(t->stop->e));
    float f = 0.f;
    APCG_HIP(hipEventElapsedTime(&f, t->start->e, t->stop->e));
    *ms = f;
    return APCG_SUCCESS;
}

// ----------------------------------------------------------------- counters

apcg_status apcg_counters_get(apcg_counters *out) {
    if (!out) return set_error(APCG_ERR_INVALID_ARG, "out is NULL");
    memset(out, 0, sizeof *out);
    out->kernel_launches = g_counters.kernel_launches.load();
    out->graph_launches = g_counters.graph_launches.load();
    out->host_syncs = g_counters.host_syncs.load();
    out->host_polls = g_counters.host_polls.load();
    out->d2h_copies = g_counters.d2h_copies.load();
    out->h2d_copies = g_counters.h2d_copies.load();
    out->stream_waits = g_counters.stream_waits.load();
    return APCG_SUCCESS;
}

apcg_status apcg_counters_reset(void) {
    g_counters.kernel_launches = 0;
    g_counters.graph_launches = 0;
    g_counters.host_syncs = 0;
    g_counters.host_polls = 0;
    g_counters.d2h_copies = 0;
    g_counters.h2d_copies = 0;
    g_counters.stream_waits = 0;
    return APCG_SUCCESS;
}

}  // extern "C"
