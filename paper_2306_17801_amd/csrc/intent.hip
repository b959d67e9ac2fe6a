// Dependency marking on arbitrary objects (Section 3.1.2, MarkIntent and
// memory registration): the caller's own work on a registered memory region
// or on a library object, enqueued on a context's stream between
// apcg_mark_intent_begin and _end, is ordered against every other access to
// that object by the same rule as the library's own operations (op_begin /
// op_end): write-write, write-read and read-write across contexts by call
// order, reads unordered, program order within a context.
#include <hip/hip_runtime.h>

#include <atomic>
#include <map>
#include <string>

#include "internal.h"

namespace apcg {
namespace {

struct Region {
    int device;
    uintptr_t start;
    int64_t bytes;
    Record rec;
};

struct Marked {
    Record *rec;       // the region's own record, or a library object's
    Region *region;    // owned when the id names a registered region
    int device;
};

// guarded by g_mu (the registry lock of every Record)
std::map<uint64_t, Marked> g_marked;
std::map<std::pair<int, uintptr_t>, uint64_t> g_regions;  // (device, start) -> id
std::atomic<uint64_t> g_next_mark{1};

}  // namespace

uint64_t intent_object_id(uint64_t *slot, int device, Record *rec) {
    std::lock_guard<std::recursive_mutex> lk(g_mu);
    if (!*slot) {
        *slot = g_next_mark++;
        g_marked[*slot] = Marked{rec, nullptr, device};
    }
    return *slot;
}

void intent_forget(uint64_t id) {
    std::lock_guard<std::recursive_mutex> lk(g_mu);
    auto it = g_marked.find(id);
    if (it == g_marked.end()) return;
    if (it->second.region) {
        g_regions.erase({it->second.region->device, it->second.region->start});
        delete it->second.region;
    }
    g_marked.erase(it);
}

}  // namespace apcg

using namespace apcg;

static bool valid_mode(int32_t m) {
    return m == APCG_ACCESS_READ || m == APCG_ACCESS_WRITE || m == APCG_ACCESS_READ_WRITE;
}

extern "C" {

apcg_status apcg_ctx_get_stream(apcg_ctx ctx, void **stream) {
    if (!ctx || !stream) return set_error(APCG_ERR_INVALID_ARG, "NULL argument");
    *stream = (void *)ctx->stream;
    return APCG_SUCCESS;
}

apcg_status apcg_memory_register(int32_t device, const void *ptr, int64_t bytes, uint64_t *id) {
    if (!ptr || bytes <= 0 || !id) return set_error(APCG_ERR_INVALID_ARG, "bad region");
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count)
        return set_error(APCG_ERR_INVALID_ARG, "no such device");
    const uintptr_t start = (uintptr_t)ptr;
    std::lock_guard<std::recursive_mutex> lk(g_mu);
    auto it = g_regions.find({device, start});
    if (it != g_regions.end()) {
        if (g_marked[it->second].region->bytes != bytes)
            return set_error(APCG_ERR_INVALID_ARG, "region already registered with another size");
        *id = it->second;
        return APCG_SUCCESS;
    }
    // no overlap with a registered region of the same device
    auto next = g_regions.lower_bound({device, start});
    if (next != g_regions.end() && next->first.first == device && next->first.second < start + (uintptr_t)bytes)
        return set_error(APCG_ERR_INVALID_ARG, "region overlaps a registered one");
    if (next != g_regions.begin()) {
        auto prev = std::prev(next);
        if (prev->first.first == device) {
            const Region *r = g_marked[prev->second].region;
            if (r->start + (uintptr_t)r->bytes > start)
                return set_error(APCG_ERR_INVALID_ARG, "region overlaps a registered one");
        }
    }
    Region *r = new Region{device, start, bytes, Record{}};
    const uint64_t nid = g_next_mark++;
    g_marked[nid] = Marked{&r->rec, r, device};
    g_regions[{device, start}] = nid;
    *id = nid;
    return APCG_SUCCESS;
}

apcg_status apcg_memory_lookup(int32_t device, const void *ptr, uint64_t *id, const void **start, int64_t *bytes) {
    if (!ptr || !id) return set_error(APCG_ERR_INVALID_ARG, "NULL argument");
    const uintptr_t p = (uintptr_t)ptr;
    std::lock_guard<std::recursive_mutex> lk(g_mu);
    auto it = g_regions.upper_bound({device, p});
    if (it != g_regions.begin()) {
        --it;
        const Region *r = g_marked[it->second].region;
        if (it->first.first == device && p >= r->start && p < r->start + (uintptr_t)r->bytes) {
            *id = it->second;
            if (start) *start = (const void *)r->start;
            if (bytes) *bytes = r->bytes;
            return APCG_SUCCESS;
        }
    }
    return set_error(APCG_ERR_INVALID_ARG, "pointer is not in a registered region");
}

apcg_status apcg_memory_unregister(uint64_t id) {
    std::lock_guard<std::recursive_mutex> lk(g_mu);
    auto it = g_marked.find(id);
    if (it == g_marked.end() || !it->second.region)
        return set_error(APCG_ERR_INVALID_ARG, "not a registered region");
    intent_forget(id);
    return APCG_SUCCESS;
}

apcg_status apcg_vec_get_id(apcg_vec v, uint64_t *id) {
    if (!v || !id) return set_error(APCG_ERR_INVALID_ARG, "NULL argument");
    *id = intent_object_id(&v->mark_id, v->device, &v->rec);
    return APCG_SUCCESS;
}

apcg_status apcg_scalar_get_id(apcg_scalar s, uint64_t *id) {
    if (!s || !id) return set_error(APCG_ERR_INVALID_ARG, "NULL argument");
    *id = intent_object_id(&s->mark_id, s->device, &s->rec);
    return APCG_SUCCESS;
}

apcg_status apcg_mat_get_id(apcg_mat A, uint64_t *id) {
    if (!A || !id) return set_error(APCG_ERR_INVALID_ARG, "NULL argument");
    *id = intent_object_id(&A->mark_id, A->device, &A->rec);
    return APCG_SUCCESS;
}

static apcg_status marked(apcg_ctx ctx, uint64_t id, int32_t mode, const char *description, Acc *acc) {
    const std::string what = description ? std::string(" (") + description + ")" : std::string();
    if (!ctx) return set_error(APCG_ERR_INVALID_ARG, "ctx is NULL" + what);
    if (!valid_mode(mode)) return set_error(APCG_ERR_INVALID_ARG, "unknown access mode" + what);
    std::lock_guard<std::recursive_mutex> lk(g_mu);
    auto it = g_marked.find(id);
    if (it == g_marked.end()) return set_error(APCG_ERR_INVALID_ARG, "unknown object id" + what);
    if (it->second.device != ctx->device)
        return set_error(APCG_ERR_INVALID_ARG, "object and context on different devices" + what);
    *acc = Acc{it->second.rec, mode == APCG_ACCESS_READ ? ACC_R : mode == APCG_ACCESS_WRITE ? ACC_W : ACC_RW};
    return APCG_SUCCESS;
}

apcg_status apcg_mark_intent_begin(apcg_ctx ctx, uint64_t id, int32_t mode, const char *description) {
    try {
        Acc acc;
        apcg_status s = marked(ctx, id, mode, description, &acc);
        if (s) return s;
        return op_begin(ctx, &acc, 1);
    } catch (const std::bad_alloc &) {
        return set_error(APCG_ERR_OUT_OF_MEMORY, "host allocation failed");
    }
}

apcg_status apcg_mark_intent_end(apcg_ctx ctx, uint64_t id, int32_t mode, const char *description) {
    try {
        Acc acc;
        apcg_status s = marked(ctx, id, mode, description, &acc);
        if (s) return s;
        return op_end(ctx, &acc, 1);
    } catch (const std::bad_alloc &) {
        return set_error(APCG_ERR_OUT_OF_MEMORY, "host allocation failed");
    }
}

}  // extern "C"
