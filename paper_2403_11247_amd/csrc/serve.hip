// Continuous-batching server for forward-only novel views of one resident
// map.  Each slot is one pass in flight: its own stream, pinned staging and
// buffers sized for max_views views of the map.  progress() retires finished
// passes and packs waiting requests, in arrival order, into free slots while
// their pair estimates fit the slot's sort buffers.  A pass is the same
// projection / depth sort / tile sort / compositing as every other render
// call, over the views of its requests (entry e = view e / n, Gaussian e % n),
// so each request's images do not depend on what it was batched with.
//
// A server created from anchors serves the view-dependent decode (eqs.
// (8)-(9)): a pass first decodes its requests' camera centres in one launch
// into the slot's stacked per-view sets, then renders each request from its
// own set (the per-view form of the same pass).
#include <algorithm>
#include <chrono>
#include <cmath>
#include <deque>
#include <sched.h>

#include "frame.h"

using namespace vcgs;

namespace {

struct Req {
    int64_t ticket;
    vcgs_camera cam;
    vcgs_pose pose;
    vcgs_images out;
    int64_t pixels;
    hipEvent_t submitted;  // recorded on the submitting stream; the pass waits for it
};

struct Slot {
    hipStream_t s = nullptr;
    hipEvent_t done = nullptr;
    Frame f;
    Work w{};
    uint32_t* flags_host = nullptr;  // pinned: pair count, overflow
    int64_t cap = 0;                 // pair capacity
    int64_t tiles_cap = 0;           // capacity of f.ranges in tiles
    std::vector<Req> reqs;
    bool busy = false;
    std::vector<void*> blocks_e, blocks_p, blocks_r;
    vcgs_gaussian_buffers set{};  // decoded per-view sets (servers created from anchors)
};

Prof& quiet_prof()
{
    static Prof p;  // never enabled: passes of different streams are not timed
    return p;
}

}  // namespace

struct vcgs_server {
    vcgs_ctx* ctx = nullptr;
    bool counted = false;  // included in ctx->servers
    vcgs_gaussians map{};  // the resident map; for a decoding server only n (Gaussians per view) is set
    bool decode = false;   // created from anchors: each pass decodes its requests' camera centres
    DecodeArgs dec{};
    vcgs_server_config cfg{};
    std::deque<Req> queue;
    std::vector<Slot> slots;
    std::deque<int64_t> ready;
    int64_t next_ticket = 0, passes = 0, reruns = 0;
    double ppp = 1.0;           // pairs-per-pixel estimate used for admission
    double typ = 1.0;           // typical pairs per pixel: sizes the tile sort's partitions
    double recent[32] = {};     // observed pairs per pixel of the last 32 passes
    int n_recent = 0;
    bool oom = false;

    // The admission estimate follows 1.25 x the largest observed pairs per
    // pixel of the last 32 passes (an underestimate only costs a rerun); the
    // typical value is their median (pairs per pixel varies several-fold with
    // the pose, so the bound would put most small views on the large sort
    // partitions).
    void observe(double obs)
    {
        recent[n_recent % 32] = obs;
        ++n_recent;
        const int m = std::min(n_recent, 32);
        double v[32];
        double mx = 0.0;
        for (int i = 0; i < m; ++i) {
            v[i] = recent[i];
            mx = std::max(mx, recent[i]);
        }
        std::nth_element(v, v + m / 2, v + m);
        ppp = std::max(1.25 * mx, 1e-3);
        typ = std::max(v[m / 2], 1e-3);
    }
    std::vector<hipEvent_t> spare_events;

    hipEvent_t event()
    {
        if (!spare_events.empty()) {
            hipEvent_t e = spare_events.back();
            spare_events.pop_back();
            return e;
        }
        hipEvent_t e = nullptr;
        if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return nullptr;
        return e;
    }

    void* dalloc(size_t bytes, std::vector<void*>& list)
    {
        void* p = ctx->dalloc.get(std::max<size_t>(bytes, 256));
        if (!p) {
            oom = true;
            return nullptr;
        }
        list.push_back(p);
        return p;
    }
    void dfree(std::vector<void*>& list)
    {
        for (void* p : list) ctx->dalloc.put(p);
        list.clear();
    }
    // (Re)allocates a slot's pair buffers; the slot must be idle.  On failure
    // the slot is left with no pair buffers (cap 0) and is not used again.
    int alloc_pairs(Slot& sl, int64_t cap)
    {
        dfree(sl.blocks_p);
        oom = false;
        sl.f.gids = static_cast<uint32_t*>(dalloc((size_t)cap * 4, sl.blocks_p));
        alloc_work_p(sl.w, cap, [&](int64_t c) { return static_cast<uint32_t*>(dalloc((size_t)c * 4, sl.blocks_p)); });
        if (oom) {
            dfree(sl.blocks_p);
            sl.cap = 0;
            return fail(VCGS_E_NOMEM, "server: pair buffers do not fit");
        }
        sl.cap = cap;
        return VCGS_OK;
    }
    int alloc_ranges(Slot& sl, int64_t tiles)
    {
        dfree(sl.blocks_r);
        oom = false;
        sl.f.ranges = static_cast<uint32_t*>(dalloc((size_t)tiles * 8, sl.blocks_r));
        if (oom) {
            sl.tiles_cap = 0;
            return fail(VCGS_E_NOMEM, "server: tile ranges do not fit");
        }
        sl.tiles_cap = tiles;
        return VCGS_OK;
    }
    int64_t estimate(const Req& r) const { return (int64_t)std::ceil((double)r.pixels * ppp); }

    // Takes waiting requests into the free slot sl and enqueues their pass; on
    // an error the requests go back to the front of the queue.
    int launch(Slot& sl)
    {
        const int rc = launch_inner(sl);
        if (rc != VCGS_OK) {
            for (auto it = sl.reqs.rbegin(); it != sl.reqs.rend(); ++it) queue.push_front(*it);
            sl.reqs.clear();
            sl.busy = false;
        }
        return rc;
    }

    int launch_inner(Slot& sl)
    {
        // admission: arrival order, while the pair estimates fit the slot's sort buffers
        sl.reqs.clear();
        int64_t est = 0, tiles = 0;
        while (!queue.empty() && (int)sl.reqs.size() < cfg.max_views) {
            const Req& r = queue.front();
            const int64_t e = estimate(r);
            if (!sl.reqs.empty() && est + e > sl.cap) break;
            est += e;
            tiles += (int64_t)((r.cam.width + kTile - 1) / kTile) * ((r.cam.height + kTile - 1) / kTile);
            sl.reqs.push_back(r);
            queue.pop_front();
        }
        const int V = (int)sl.reqs.size();
        if (tiles > sl.tiles_cap) {
            int rc = alloc_ranges(sl, tiles + tiles / 4);
            if (rc != VCGS_OK) return rc;
        }
        vcgs_camera cams[kMaxViews];
        vcgs_pose poses[kMaxViews];
        int64_t pix = 0;
        for (int v = 0; v < V; ++v) {
            pix += sl.reqs[v].pixels;
            cams[v] = sl.reqs[v].cam;
            poses[v] = sl.reqs[v].pose;
        }
        Frame& f = sl.f;
        build_tables(V, map.n, cams, poses, cfg.bg, f);
        vcgs_gaussians g = map;
        if (decode) {
            // x_c = -R^T t in binary64 from the pose's values, rounded to binary32
            dec.views = V;
            for (int v = 0; v < V; ++v)
                for (int i = 0; i < 3; ++i) {
                    const float* R = poses[v].R;
                    const float* t = poses[v].t;
                    dec.cam[v][i] = (float)-((double)R[i] * t[0] + (double)R[3 + i] * t[1] + (double)R[6 + i] * t[2]);
                }
            g.mean = sl.set.mean;
            g.scale = sl.set.scale;
            g.quat = sl.set.quat;
            g.opacity = sl.set.opacity;
            g.color = sl.set.color;
            f.pt.per_view = 1;
        }
        for (int v = 0; v < V; ++v) {
            f.vt.color[v] = sl.reqs[v].out.color;
            f.vt.depth[v] = sl.reqs[v].out.depth;
            f.vt.alpha[v] = sl.reqs[v].out.alpha;
        }
        // grids of the pair stages are sized from the capacity: use the pass's own
        // estimate (with a margin) rather than the whole slot
        f.cap = std::min<int64_t>(sl.cap, est + est / 4 + 4096);
        // the tile sort sizes its partitions for the typical count
        f.pair_hint = std::min<int64_t>(f.cap, (int64_t)std::ceil((double)pix * typ));
        // order the pass after whatever each request's submitting stream had
        // enqueued; an event that has already completed needs no wait
        for (const Req& r : sl.reqs)
            if (hipEventQuery(r.submitted) != hipSuccess) HIP_TRY(hipStreamWaitEvent(sl.s, r.submitted, 0));
        // the projection takes the table as a kernel argument (no upload)
        f.tab_by_value = true;
        if (f.E > 0) {
            if (decode) launch_decode_fwd(dec, sl.set, sl.s);
            const uint32_t* ord = phase_a(quiet_prof(), g, f, sl.w, sl.s);
            // the compositing launch writes the pair total and overflow flag
            // (adjacent words) into the slot's pinned words: no copy after it
            f.vt.flags_out = sl.flags_host;
            f.vt.flags_src = sl.w.total;
            phase_b(quiet_prof(), f, sl.w, ord, sl.s);
            f.vt.flags_out = nullptr;
        } else {
            f.cap = 0;
            zero_pass(f, sl.w, sl.s);
            phase_b(quiet_prof(), f, sl.w, nullptr, sl.s);  // background images
            sl.flags_host[0] = sl.flags_host[1] = 0u;
        }
        HIP_TRY(hipEventRecord(sl.done, sl.s));
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return fail(VCGS_E_HIP, std::string("server: kernel launch failed: ") + hipGetErrorString(e));
        sl.busy = true;
        ++passes;
        return VCGS_OK;
    }

    int finish(Slot& sl)
    {
        sl.busy = false;
        const int64_t total = sl.flags_host[0];
        if (sl.flags_host[1] != 0u) {
            // overflow: grow the slot, raise the estimate, rerun these requests first
            int64_t pix = 0;
            for (const Req& r : sl.reqs) pix += r.pixels;
            observe((double)total / (double)std::max<int64_t>(pix, 1));
            ++reruns;
            for (auto it = sl.reqs.rbegin(); it != sl.reqs.rend(); ++it) queue.push_front(*it);
            sl.reqs.clear();
            if (total > kMaxSortItems) return fail(VCGS_E_UNSUPPORTED, "server: a pass needs more than 2^30-1 pairs");
            if (total + total / 8 + 4096 > sl.cap)
                return alloc_pairs(sl, std::min<int64_t>(total + total / 8 + 4096, kMaxSortItems));
            return VCGS_OK;
        }
        int64_t pix = 0;
        for (const Req& r : sl.reqs) {
            ready.push_back(r.ticket);
            spare_events.push_back(r.submitted);
            pix += r.pixels;
        }
        if (pix > 0) observe((double)total / (double)pix);
        sl.reqs.clear();
        return VCGS_OK;
    }

    void release()
    {
        if (counted) {
            --ctx->servers;
            counted = false;
        }
        for (Slot& sl : slots) {
            if (sl.s) (void)hipStreamSynchronize(sl.s);
            dfree(sl.blocks_e);
            dfree(sl.blocks_p);
            dfree(sl.blocks_r);
            if (sl.flags_host) (void)hipHostFree(sl.flags_host);
            if (sl.done) (void)hipEventDestroy(sl.done);
            if (sl.s) (void)hipStreamDestroy(sl.s);
        }
        slots.clear();
        for (const Req& r : queue) spare_events.push_back(r.submitted);
        queue.clear();
        for (hipEvent_t e : spare_events) (void)hipEventDestroy(e);
        spare_events.clear();
    }
};

extern "C" {

}  // extern "C"

namespace {

// Shared by both constructors: dec is NULL for a resident map, else the
// decode of the anchors behind map (only map->n is used then).
int create_server(vcgs_ctx* ctx, const vcgs_gaussians* map, const DecodeArgs* dec, const vcgs_server_config* cfg,
                  vcgs_server** out)
{
    HIP_TRY(hipSetDevice(ctx->device));
    vcgs_server* srv = new vcgs_server();
    srv->ctx = ctx;
    ++ctx->servers;
    srv->counted = true;
    srv->map = *map;
    if (dec) {
        srv->decode = true;
        srv->dec = *dec;
    }
    srv->cfg = *cfg;
    srv->ppp = cfg->pairs_per_pixel;
    srv->typ = cfg->pairs_per_pixel;
    srv->slots.resize(cfg->slots);
    const int64_t Emax = (int64_t)cfg->max_views * map->n;
    for (Slot& sl : srv->slots) {
        bool ok = hipStreamCreateWithFlags(&sl.s, hipStreamNonBlocking) == hipSuccess &&
                  hipEventCreateWithFlags(&sl.done, hipEventDisableTiming) == hipSuccess &&
                  hipHostMalloc((void**)&sl.flags_host, 16, hipHostMallocDefault) == hipSuccess;
        if (!ok) {
            srv->release();
            delete srv;
            return fail(VCGS_E_HIP, "server: stream, event or pinned allocation failed");
        }
        Frame& f = sl.f;
        f.pt_dev = static_cast<ProjTab*>(srv->dalloc(sizeof(ProjTab), sl.blocks_e));
        f.rec = static_cast<Splat*>(srv->dalloc((size_t)Emax * sizeof(Splat), sl.blocks_e));
        f.depth_key = static_cast<uint32_t*>(srv->dalloc((size_t)Emax * 4, sl.blocks_e));
        f.rect = static_cast<uint2*>(srv->dalloc((size_t)Emax * 8, sl.blocks_e));
        f.count = static_cast<uint32_t*>(srv->dalloc((size_t)Emax * 4, sl.blocks_e));
        alloc_work_e(sl.w, Emax, [&](int64_t c) { return static_cast<uint32_t*>(srv->dalloc((size_t)c * 4, sl.blocks_e)); });
        if (dec) {  // stacked per-view sets: mean/scale/color [V][3][n], quat [V][4][n], opacity [V][n]
            sl.set.mean = static_cast<float*>(srv->dalloc((size_t)Emax * 3 * 4, sl.blocks_e));
            sl.set.scale = static_cast<float*>(srv->dalloc((size_t)Emax * 3 * 4, sl.blocks_e));
            sl.set.quat = static_cast<float*>(srv->dalloc((size_t)Emax * 4 * 4, sl.blocks_e));
            sl.set.opacity = static_cast<float*>(srv->dalloc((size_t)Emax * 4, sl.blocks_e));
            sl.set.color = static_cast<float*>(srv->dalloc((size_t)Emax * 3 * 4, sl.blocks_e));
        }
        if (srv->oom || srv->alloc_pairs(sl, cfg->pair_budget) != VCGS_OK || srv->alloc_ranges(sl, 4096) != VCGS_OK) {
            srv->release();
            delete srv;
            return fail(VCGS_E_NOMEM, "server: slot buffers do not fit");
        }
    }
    *out = srv;
    return VCGS_OK;
}

int check_config(const vcgs_server_config* cfg)
{
    if (cfg->max_views < 1 || cfg->max_views > kMaxViews) return fail(VCGS_E_INVALID, "max_views must be in [1, 16]");
    if (cfg->slots < 1 || cfg->slots > 8) return fail(VCGS_E_INVALID, "slots must be in [1, 8]");
    if (cfg->pair_budget <= 0 || !(cfg->pairs_per_pixel > 0.0f))
        return fail(VCGS_E_INVALID, "pair_budget and pairs_per_pixel must be positive");
    if (cfg->pair_budget > kMaxSortItems) return fail(VCGS_E_UNSUPPORTED, "pair_budget above 2^30-1");
    return VCGS_OK;
}

}  // namespace

extern "C" {

int vcgs_server_create(vcgs_ctx* ctx, const vcgs_gaussians* map, const vcgs_server_config* cfg, vcgs_server** out)
{
    if (!ctx || !cfg || !out) return fail(VCGS_E_INVALID, "ctx, cfg or out is NULL");
    *out = nullptr;
    int rc;
    if ((rc = check_config(cfg)) != VCGS_OK) return rc;
    if ((rc = check_gaussians(map, cfg->max_views)) != VCGS_OK) return rc;
    return create_server(ctx, map, nullptr, cfg, out);
}

int vcgs_server_create_anchors(vcgs_ctx* ctx, const vcgs_anchors* a, const vcgs_mlp* mlp, const vcgs_codebook* cb,
                               const float* mask_logit, float mask_eps, const vcgs_server_config* cfg,
                               vcgs_server** out)
{
    if (!ctx || !cfg || !out) return fail(VCGS_E_INVALID, "ctx, cfg or out is NULL");
    *out = nullptr;
    int rc;
    if ((rc = check_config(cfg)) != VCGS_OK) return rc;
    DecodeArgs d;
    const float origin[3] = {0.0f, 0.0f, 0.0f};  // placeholder centre: each pass sets its own
    if ((rc = make_decode_args(a, mlp, cb, mask_logit, mask_eps, &d, origin, 1)) != VCGS_OK) return rc;
    if (d.na * d.k * (int64_t)cfg->max_views > kMaxSortItems)
        return fail(VCGS_E_UNSUPPORTED, "server: max_views x Gaussians above 2^30-1");
    vcgs_gaussians map{};
    map.n = d.na * d.k;
    return create_server(ctx, &map, &d, cfg, out);
}

void vcgs_server_destroy(vcgs_server* srv)
{
    if (!srv) return;
    (void)hipSetDevice(srv->ctx->device);
    srv->release();
    delete srv;
}

int vcgs_server_submit(vcgs_server* srv, const vcgs_camera* cam, const vcgs_pose* pose, const vcgs_images* out,
                       int64_t* ticket, void* stream)
{
    if (!srv || !pose || !out) return fail(VCGS_E_INVALID, "srv, pose or out is NULL");
    int rc;
    if ((rc = check_camera(cam)) != VCGS_OK) return rc;
    if (!out->color || !out->depth || !out->alpha) return fail(VCGS_E_INVALID, "an output image is NULL");
    Req r;
    r.ticket = srv->next_ticket++;
    r.cam = *cam;
    r.pose = *pose;
    r.out = *out;
    r.pixels = (int64_t)cam->width * cam->height;
    HIP_TRY(hipSetDevice(srv->ctx->device));
    r.submitted = srv->event();
    if (!r.submitted) return fail(VCGS_E_HIP, "server: event creation failed");
    if (hipEventRecord(r.submitted, (hipStream_t)stream) != hipSuccess) {
        srv->spare_events.push_back(r.submitted);
        return fail(VCGS_E_HIP, "server: event record failed");
    }
    srv->queue.push_back(r);
    if (ticket) *ticket = r.ticket;
    return VCGS_OK;
}

int vcgs_server_progress(vcgs_server* srv, int64_t timeout_us, int64_t* done, int32_t max_done, int32_t* n_done)
{
    if (!srv || !n_done || (max_done > 0 && !done)) return fail(VCGS_E_INVALID, "srv, done or n_done is NULL");
    *n_done = 0;
    HIP_TRY(hipSetDevice(srv->ctx->device));
    const auto t0 = std::chrono::steady_clock::now();
    for (;;) {
        bool moved = false;
        for (Slot& sl : srv->slots) {
            if (!sl.busy) continue;
            const hipError_t q = hipEventQuery(sl.done);
            if (q == hipErrorNotReady) continue;
            if (q != hipSuccess) return fail(VCGS_E_HIP, std::string("server: pass failed: ") + hipGetErrorString(q));
            int rc = srv->finish(sl);
            if (rc != VCGS_OK) return rc;
            moved = true;
        }
        for (Slot& sl : srv->slots) {
            if (srv->queue.empty()) break;
            if (sl.busy || sl.cap == 0) continue;  // cap 0: a failed resize retired the slot
            int rc = srv->launch(sl);
            if (rc != VCGS_OK) return rc;
            moved = true;
        }
        bool usable = false;
        for (const Slot& sl : srv->slots) usable = usable || sl.cap > 0;
        if (!usable) return fail(VCGS_E_NOMEM, "server: no slot has pair buffers left");
        while (!srv->ready.empty() && *n_done < max_done) {
            done[(*n_done)++] = srv->ready.front();
            srv->ready.pop_front();
        }
        if (moved || *n_done > 0) return VCGS_OK;
        const auto us = std::chrono::duration_cast<std::chrono::microseconds>(std::chrono::steady_clock::now() - t0);
        if (us.count() >= timeout_us) return VCGS_OK;
        sched_yield();
    }
}

int vcgs_server_stats_read(const vcgs_server* srv, vcgs_server_stats* out)
{
    if (!srv || !out) return fail(VCGS_E_INVALID, "srv or out is NULL");
    out->queued = (int64_t)srv->queue.size();
    out->in_flight = 0;
    for (const Slot& sl : srv->slots) out->in_flight += sl.busy ? 1 : 0;
    out->passes = srv->passes;
    out->reruns = srv->reruns;
    out->pairs_per_pixel = (float)srv->ppp;
    return VCGS_OK;
}

}  // extern "C"
