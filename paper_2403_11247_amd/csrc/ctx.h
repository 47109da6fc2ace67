// Context, device memory pool and stage timers shared by the library's
// translation units.
#pragma once

#include <algorithm>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "internal.h"

namespace vcgs {

extern thread_local std::string g_err;

inline int fail(int code, const std::string& msg)
{
    g_err = msg;
    return code;
}

#define HIP_TRY(expr)                                                                                 \
    do {                                                                                              \
        hipError_t e_ = (expr);                                                                       \
        if (e_ != hipSuccess) return ::vcgs::fail(VCGS_E_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

// Where device memory comes from: hipMalloc / hipFree, or the caller's
// functions (vcgs_set_allocator), e.g. a framework's caching allocator.
struct DevAlloc {
    void* (*alloc_fn)(size_t, void*) = nullptr;
    void (*free_fn)(void*, void*) = nullptr;
    void* user = nullptr;
    void* get(size_t bytes)
    {
        if (alloc_fn) return alloc_fn(bytes, user);
        void* p = nullptr;
        if (hipMalloc(&p, bytes) != hipSuccess) {
            (void)hipGetLastError();
            return nullptr;
        }
        return p;
    }
    void put(void* p)
    {
        if (!p) return;
        if (free_fn)
            free_fn(p, user);
        else
            (void)hipFree(p);
    }
};

// Caching allocator.  Blocks freed by the library go back to a size-keyed
// free list and are reused by later requests; all work of a context is
// ordered on the caller's stream, so a block released by one call is only
// touched again by work enqueued after it.
struct Pool {
    DevAlloc* dev = nullptr;  // the context's source of device memory
    std::multimap<size_t, void*> free_blocks;
    std::map<void*, size_t> sizes;
    size_t cached = 0;

    static size_t round_up(size_t n)
    {
        if (n < 4096) return 4096;
        size_t p = 1;
        while (p < n) p <<= 1;
        const size_t step = p >> 3;  // 1/8 of the next power of two
        return (n + step - 1) / step * step;
    }

    void* alloc(size_t bytes)
    {
        const size_t want = round_up(bytes);
        auto it = free_blocks.lower_bound(want);
        if (it != free_blocks.end() && it->first <= 2 * want) {
            void* p = it->second;
            cached -= it->first;
            free_blocks.erase(it);
            return p;
        }
        void* p = dev->get(want);
        if (!p) {
            release_cache();
            p = dev->get(want);
            if (!p) return nullptr;
        }
        sizes[p] = want;
        return p;
    }

    void free(void* p)
    {
        if (!p) return;
        auto it = sizes.find(p);
        if (it == sizes.end()) return;
        free_blocks.emplace(it->second, p);
        cached += it->second;
    }

    void release_cache()
    {
        if (free_blocks.empty()) return;
        (void)hipDeviceSynchronize();
        for (auto& kv : free_blocks) {
            dev->put(kv.second);
            sizes.erase(kv.second);
        }
        free_blocks.clear();
        cached = 0;
    }

    void destroy()
    {
        (void)hipDeviceSynchronize();
        for (auto& kv : sizes) dev->put(kv.first);
        sizes.clear();
        free_blocks.clear();
        cached = 0;
    }
};

// Scoped group of pool blocks released together.
struct Scratch {
    Pool* pool;
    std::vector<void*> blocks;
    bool oom = false;
    explicit Scratch(Pool* p) : pool(p) {}
    ~Scratch()
    {
        for (void* b : blocks) pool->free(b);
    }
    template <class T>
    T* get(int64_t count)
    {
        void* p = pool->alloc((size_t)std::max<int64_t>(count, 1) * sizeof(T));
        if (!p) oom = true;
        blocks.push_back(p);
        return static_cast<T*>(p);
    }
};


// Per-stage HIP-event timing on the caller's stream.
struct Prof {
    bool on = false;
    uint32_t mask = 0xFFFFu;  // stages timed while on (bit = stage)
    bool count = false;
    bool capturing = false;  // a graph is being captured: record nothing
    struct Rec {
        int stage;
        hipEvent_t a, b;
    };
    std::vector<Rec> pending;
    std::vector<hipEvent_t> spare;
    double ms[VCGS_STAGE_COUNT] = {};
    int64_t launches[VCGS_STAGE_COUNT] = {};
    unsigned long long* d_counters = nullptr;  // 5 x u64 on the device

    hipEvent_t event()
    {
        if (!spare.empty()) {
            hipEvent_t e = spare.back();
            spare.pop_back();
            return e;
        }
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        return e;
    }
    void begin(int stage, hipStream_t s)
    {
        if (!on || capturing || !((mask >> stage) & 1u)) return;
        if (pending.size() > 8192) fold();
        Rec r{stage, event(), event()};
        if (r.a) (void)hipEventRecord(r.a, s);
        pending.push_back(r);
    }
    void end(int stage, hipStream_t s)
    {
        if (!on || capturing || !((mask >> stage) & 1u)) return;
        for (auto it = pending.rbegin(); it != pending.rend(); ++it)
            if (it->stage == stage) {
                if (it->b) (void)hipEventRecord(it->b, s);
                return;
            }
    }
    void fold()
    {
        for (auto& r : pending) {
            float t = 0.0f;
            if (r.a && r.b && hipEventSynchronize(r.b) == hipSuccess && hipEventElapsedTime(&t, r.a, r.b) == hipSuccess) {
                ms[r.stage] += t;
                launches[r.stage] += 1;
            }
            if (r.a) spare.push_back(r.a);
            if (r.b) spare.push_back(r.b);
        }
        pending.clear();
    }
    void clear()
    {
        fold();
        for (int i = 0; i < VCGS_STAGE_COUNT; ++i) { ms[i] = 0.0; launches[i] = 0; }
    }
    void destroy()
    {
        fold();
        for (hipEvent_t e : spare) (void)hipEventDestroy(e);
        spare.clear();
    }
};


struct BatchPlan;

}  // namespace vcgs

struct vcgs_ctx {
    int device = 0;
    vcgs::DevAlloc dalloc;
    vcgs::Pool pool;  // pool.dev = &dalloc
    vcgs::Prof prof;
    uint32_t* host_u32 = nullptr;  // pinned readback slot
    vcgs::ProjTab* host_tab = nullptr;  // pinned staging of the per-view table
    hipStream_t graph_stream = nullptr;  // stream that captures and replays graphs
    hipEvent_t graph_done = nullptr;
    std::vector<vcgs::BatchPlan*> plans;  // prepared batched windows, most recent last
    vcgs::BatchPlan* last_plan = nullptr;
    hipStream_t last_stream = nullptr;
    vcgs::BatchPlan* fwd_plan = nullptr;  // last forward kept for vcgs_render_batch_backward
    int64_t last_required_pairs = 0;      // pair count of the last pass that outgrew its buffers
    int servers = 0;  // live servers (their slot buffers come from dalloc)
};

namespace vcgs {
void destroy_plans(vcgs_ctx* ctx);
// Device address of the allocation-free forward's scratch array on `device`
// (which must be current); looked up once per device.
int noalloc_init(int device);
}  // namespace vcgs
