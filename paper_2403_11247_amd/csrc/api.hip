// C ABI of the vcgs library: contexts, device memory, saved states, and the
// order of kernels for the forward and backward render and the decode.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "internal.h"

using namespace vcgs;

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg)
{
    g_err = msg;
    return code;
}

#define HIP_TRY(expr)                                                                       \
    do {                                                                                    \
        hipError_t e_ = (expr);                                                             \
        if (e_ != hipSuccess) return fail(VCGS_E_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

// Caching allocator.  Blocks freed by the library go back to a size-keyed
// free list and are reused by later requests; all work of a context is
// ordered on the caller's stream, so a block released by one call is only
// touched again by work enqueued after it.
struct Pool {
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
        void* p = nullptr;
        if (hipMalloc(&p, want) != hipSuccess) {
            (void)hipGetLastError();
            release_cache();
            if (hipMalloc(&p, want) != hipSuccess) {
                (void)hipGetLastError();
                return nullptr;
            }
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
            (void)hipFree(kv.second);
            sizes.erase(kv.second);
        }
        free_blocks.clear();
        cached = 0;
    }

    void destroy()
    {
        (void)hipDeviceSynchronize();
        for (auto& kv : sizes) (void)hipFree(kv.first);
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

}  // namespace

// Per-stage HIP-event timing on the caller's stream.
struct Prof {
    bool on = false;
    bool count = false;
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
        if (!on) return;
        if (pending.size() > 8192) fold();
        Rec r{stage, event(), event()};
        if (r.a) (void)hipEventRecord(r.a, s);
        pending.push_back(r);
    }
    void end(int stage, hipStream_t s)
    {
        if (!on) return;
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

struct vcgs_ctx {
    int device = 0;
    Pool pool;
    Prof prof;
    uint32_t* host_u32 = nullptr;  // pinned readback slot
};

struct vcgs_state {
    vcgs_ctx* ctx = nullptr;
    int64_t n = 0, P = 0;
    int W = 0, H = 0, tiles_x = 0, tiles_y = 0;
    float bg[3] = {0, 0, 0};
    Splat* rec = nullptr;
    uint32_t* depth_key = nullptr;
    uint2* rect = nullptr;
    uint32_t* count = nullptr;
    uint32_t* gids = nullptr;
    uint32_t* ranges = nullptr;
    float* t_final = nullptr;
    uint32_t* n_contrib = nullptr;
    std::vector<void*> blocks;

    template <class T>
    T* get(int64_t count_)
    {
        void* p = ctx->pool.alloc((size_t)std::max<int64_t>(count_, 1) * sizeof(T));
        blocks.push_back(p);
        return static_cast<T*>(p);
    }
    bool ok() const
    {
        for (void* b : blocks)
            if (!b) return false;
        return true;
    }
    void release()
    {
        for (void* b : blocks) ctx->pool.free(b);
        blocks.clear();
    }
};

namespace {

int check_camera(const vcgs_camera* c)
{
    if (!c) return fail(VCGS_E_INVALID, "camera is NULL");
    if (c->width <= 0 || c->height <= 0) return fail(VCGS_E_INVALID, "camera width/height must be positive");
    if (c->width > 65535 * kTile || c->height > 65535 * kTile) return fail(VCGS_E_UNSUPPORTED, "image too large");
    if (c->tile != kTile) return fail(VCGS_E_INVALID, "camera tile must be 16");
    if (!(c->fx > 0.0f) || !(c->fy > 0.0f)) return fail(VCGS_E_INVALID, "focal lengths must be positive");
    return VCGS_OK;
}

int check_gaussians(const vcgs_gaussians* g)
{
    if (!g) return fail(VCGS_E_INVALID, "gaussians is NULL");
    if (g->n < 0) return fail(VCGS_E_INVALID, "negative Gaussian count");
    if (g->n >= (int64_t)1 << 31) return fail(VCGS_E_UNSUPPORTED, "at most 2^31-1 Gaussians");
    if (g->n > 0 && (!g->mean || !g->scale || !g->quat || !g->opacity || !g->color))
        return fail(VCGS_E_INVALID, "a Gaussian attribute pointer is NULL");
    return VCGS_OK;
}

int bits_for(uint32_t v)
{
    int b = 1;
    while (b < 32 && (v >> b) != 0u) ++b;
    return b;
}

}  // namespace

extern "C" {

const char* vcgs_last_error(void) { return g_err.c_str(); }
const char* vcgs_version(void) { return "vcgs 0.1 gfx950"; }

int vcgs_create(int device, vcgs_ctx** out)
{
    if (!out) return fail(VCGS_E_INVALID, "out is NULL");
    *out = nullptr;
    int count = 0;
    HIP_TRY(hipGetDeviceCount(&count));
    if (device < 0 || device >= count) return fail(VCGS_E_INVALID, "no such HIP device");
    hipDeviceProp_t prop;
    HIP_TRY(hipGetDeviceProperties(&prop, device));
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return fail(VCGS_E_UNSUPPORTED, std::string("device is ") + prop.gcnArchName + ", not gfx950");
    HIP_TRY(hipSetDevice(device));
    vcgs_ctx* c = new vcgs_ctx();
    c->device = device;
    if (hipHostMalloc((void**)&c->host_u32, 64, hipHostMallocDefault) != hipSuccess) {
        delete c;
        return fail(VCGS_E_NOMEM, "pinned host allocation failed");
    }
    *out = c;
    return VCGS_OK;
}

void vcgs_destroy(vcgs_ctx* ctx)
{
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    ctx->prof.destroy();
    if (ctx->prof.d_counters) (void)hipFree(ctx->prof.d_counters);
    ctx->pool.destroy();
    if (ctx->host_u32) (void)hipHostFree(ctx->host_u32);
    delete ctx;
}

void vcgs_state_free(vcgs_ctx* ctx, vcgs_state* st)
{
    (void)ctx;
    if (!st) return;
    st->release();
    delete st;
}

int vcgs_state_query(const vcgs_state* st, vcgs_state_view* out)
{
    if (!st || !out) return fail(VCGS_E_INVALID, "NULL argument");
    out->n = st->n;
    out->n_pairs = st->P;
    out->tiles_x = st->tiles_x;
    out->tiles_y = st->tiles_y;
    out->depth_bits = st->depth_key;
    out->rect = reinterpret_cast<const uint16_t*>(st->rect);
    out->count = st->count;
    out->gids = st->gids;
    out->ranges = st->ranges;
    out->t_final = st->t_final;
    out->n_contrib = st->n_contrib;
    out->splats = reinterpret_cast<const float*>(st->rec);
    return VCGS_OK;
}

int vcgs_render_forward(vcgs_ctx* ctx, const vcgs_gaussians* g, const vcgs_camera* cam, const vcgs_pose* pose,
                        const float bg[3], vcgs_images* out, vcgs_state** state_out, void* stream)
{
    if (!ctx) return fail(VCGS_E_INVALID, "ctx is NULL");
    int rc;
    if ((rc = check_gaussians(g)) != VCGS_OK) return rc;
    if ((rc = check_camera(cam)) != VCGS_OK) return rc;
    if (!pose || !bg || !out || !out->color || !out->depth || !out->alpha)
        return fail(VCGS_E_INVALID, "pose, bg or an output image is NULL");
    if (state_out) *state_out = nullptr;
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(hipSetDevice(ctx->device));

    const int64_t n = g->n;
    const CamK ck = make_camk(*cam);
    const PoseK pk = make_posek(*pose);
    const uint32_t n_tiles = (uint32_t)(ck.tiles_x * ck.tiles_y);
    const int64_t HW = (int64_t)cam->width * cam->height;

    vcgs_state* st = new vcgs_state();
    st->ctx = ctx;
    st->n = n;
    st->W = cam->width;
    st->H = cam->height;
    st->tiles_x = ck.tiles_x;
    st->tiles_y = ck.tiles_y;
    for (int i = 0; i < 3; ++i) st->bg[i] = bg[i];
    st->rec = st->get<Splat>(n);
    st->depth_key = st->get<uint32_t>(n);
    st->rect = st->get<uint2>(n);
    st->count = st->get<uint32_t>(n);
    st->ranges = st->get<uint32_t>(2 * (int64_t)n_tiles);
    st->t_final = st->get<float>(HW);
    st->n_contrib = st->get<uint32_t>(HW);
    auto drop = [&](int code, const std::string& m) {
        st->release();
        delete st;
        return fail(code, m);
    };
    if (!st->ok()) return drop(VCGS_E_NOMEM, "device allocation failed (state)");

    int64_t P = 0;
    {
        Scratch sc(&ctx->pool);
        Prof& pf = ctx->prof;
        pf.begin(VCGS_STAGE_PREPROCESS, s);
        launch_preprocess(n, *g, ck, pk, st->rec, st->depth_key, st->rect, st->count, s);
        pf.end(VCGS_STAGE_PREPROCESS, s);
        if (n > 0) {
            // depth order of all Gaussians (culled ones carry the largest key and end up last)
            const int nb = radix_blocks(n);
            uint32_t* dk = sc.get<uint32_t>(n);
            uint32_t* order = sc.get<uint32_t>(n);
            SortTemp t;
            t.keys_alt = sc.get<uint32_t>(n);
            t.vals_alt = sc.get<uint32_t>(n);
            t.hist = sc.get<uint32_t>((int64_t)256 * nb);
            t.scan_tmp = sc.get<uint32_t>(scan_temp_words((int64_t)256 * nb) + scan_temp_words(n) + 8);
            uint32_t* cnt_sorted = sc.get<uint32_t>(n);
            uint32_t* offs = sc.get<uint32_t>(n);
            uint32_t* d_total = sc.get<uint32_t>(4);
            if (sc.oom) return drop(VCGS_E_NOMEM, "device allocation failed (depth sort)");
            pf.begin(VCGS_STAGE_DEPTH_SORT, s);
            if (hipMemcpyAsync(dk, st->depth_key, n * sizeof(uint32_t), hipMemcpyDeviceToDevice, s) != hipSuccess)
                return drop(VCGS_E_HIP, "hipMemcpyAsync failed");
            const int which = radix_sort_u32(dk, order, true, n, 32, t, s);
            pf.end(VCGS_STAGE_DEPTH_SORT, s);
            const uint32_t* ord = which ? t.vals_alt : order;
            pf.begin(VCGS_STAGE_PAIR_SCAN, s);
            launch_gather_counts(n, ord, st->count, cnt_sorted, s);
            exclusive_scan_u32(cnt_sorted, offs, n, d_total, t.scan_tmp, s);
            pf.end(VCGS_STAGE_PAIR_SCAN, s);
            if (hipMemcpyAsync(ctx->host_u32, d_total, sizeof(uint32_t), hipMemcpyDeviceToHost, s) != hipSuccess ||
                hipStreamSynchronize(s) != hipSuccess)
                return drop(VCGS_E_HIP, std::string("pair count readback failed: ") + hipGetErrorString(hipGetLastError()));
            P = ctx->host_u32[0];
            st->P = P;
            st->gids = st->get<uint32_t>(P);
            if (!st->ok()) return drop(VCGS_E_NOMEM, "device allocation failed (pairs)");
            launch_fill_u32(st->ranges, 0u, 2 * (int64_t)n_tiles, s);
            if (P > 0) {
                const int nbp = radix_blocks(P);
                uint32_t* tile_ids = sc.get<uint32_t>(P);
                SortTemp tp;
                tp.keys_alt = sc.get<uint32_t>(P);
                tp.vals_alt = sc.get<uint32_t>(P);
                tp.hist = sc.get<uint32_t>((int64_t)256 * nbp);
                tp.scan_tmp = sc.get<uint32_t>(scan_temp_words((int64_t)256 * nbp) + 8);
                if (sc.oom) return drop(VCGS_E_NOMEM, "device allocation failed (pair sort)");
                pf.begin(VCGS_STAGE_EMIT, s);
                launch_emit_pairs(n, ord, offs, st->count, st->rect, ck.tiles_x, 0u, tile_ids, st->gids, s);
                pf.end(VCGS_STAGE_EMIT, s);
                pf.begin(VCGS_STAGE_TILE_SORT, s);
                const int w = radix_sort_u32(tile_ids, st->gids, false, P, bits_for(n_tiles - 1), tp, s);
                const uint32_t* tsorted = w ? tp.keys_alt : tile_ids;
                if (w) {
                    if (hipMemcpyAsync(st->gids, tp.vals_alt, P * sizeof(uint32_t), hipMemcpyDeviceToDevice, s) !=
                        hipSuccess)
                        return drop(VCGS_E_HIP, "hipMemcpyAsync failed");
                }
                pf.end(VCGS_STAGE_TILE_SORT, s);
                pf.begin(VCGS_STAGE_TILE_RANGES, s);
                launch_tile_ranges(P, tsorted, n_tiles, st->ranges, s);
                pf.end(VCGS_STAGE_TILE_RANGES, s);
            }
        } else {
            launch_fill_u32(st->ranges, 0u, 2 * (int64_t)n_tiles, s);
        }
        unsigned long long* cnts = nullptr;
        if (pf.count && pf.d_counters) {
            cnts = pf.d_counters;
            launch_fill_u32(reinterpret_cast<uint32_t*>(cnts), 0u, 4, s);
        }
        pf.begin(VCGS_STAGE_COMPOSITE, s);
        launch_composite_fwd(ck, st->rec, st->gids, st->ranges, st->bg, out->color, out->depth, out->alpha,
                             st->t_final, st->n_contrib, cnts, s);
        pf.end(VCGS_STAGE_COMPOSITE, s);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return drop(VCGS_E_HIP, std::string("kernel launch failed: ") + hipGetErrorString(e));
    }
    if (state_out) {
        *state_out = st;
    } else {
        st->release();
        delete st;
    }
    return VCGS_OK;
}

int vcgs_render_backward(vcgs_ctx* ctx, const vcgs_state* st, const vcgs_gaussians* g, const vcgs_camera* cam,
                         const vcgs_pose* pose, const float* dl_dcolor, const float* dl_ddepth,
                         const float* dl_dalpha, vcgs_gaussian_buffers* grads, float* dl_dpose, void* stream)
{
    if (!ctx || !st) return fail(VCGS_E_INVALID, "ctx or state is NULL");
    int rc;
    if ((rc = check_gaussians(g)) != VCGS_OK) return rc;
    if ((rc = check_camera(cam)) != VCGS_OK) return rc;
    if (!pose) return fail(VCGS_E_INVALID, "pose is NULL");
    if (g->n != st->n || cam->width != st->W || cam->height != st->H)
        return fail(VCGS_E_INVALID, "Gaussians or camera differ from the forward call");
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(hipSetDevice(ctx->device));
    const int64_t n = g->n;
    const CamK ck = make_camk(*cam);
    const PoseK pk = make_posek(*pose);
    vcgs_gaussian_buffers gb = grads ? *grads : vcgs_gaussian_buffers{nullptr, nullptr, nullptr, nullptr, nullptr};
    Scratch sc(&ctx->pool);
    const int pb = std::max(1, preprocess_bwd_blocks(n));
    float* g2 = sc.get<float>((int64_t)kG2 * n);
    float* partial = sc.get<float>(6 * (int64_t)pb);
    if (sc.oom) return fail(VCGS_E_NOMEM, "device allocation failed (backward)");
    Prof& pf = ctx->prof;
    unsigned long long* cnts = nullptr;
    if (pf.count && pf.d_counters) {
        cnts = pf.d_counters;
        launch_fill_u32(reinterpret_cast<uint32_t*>(cnts) + 4, 0u, 6, s);
    }
    launch_fill_f32(g2, 0.0f, (int64_t)kG2 * n, s);
    pf.begin(VCGS_STAGE_COMPOSITE_BWD, s);
    if (n > 0 && st->P > 0)
        launch_composite_bwd(ck, st->rec, st->gids, st->ranges, st->bg, st->t_final, st->n_contrib, dl_dcolor,
                             dl_ddepth, dl_dalpha, g2, cnts, s);
    pf.end(VCGS_STAGE_COMPOSITE_BWD, s);
    pf.begin(VCGS_STAGE_PREPROCESS_BWD, s);
    if (n > 0)
        launch_preprocess_bwd(n, *g, ck, pk, st->count, g2, gb, partial, pb, s);
    else
        launch_fill_f32(partial, 0.0f, 6, s);
    if (dl_dpose) launch_pose_reduce(partial, n > 0 ? pb : 1, dl_dpose, s);
    pf.end(VCGS_STAGE_PREPROCESS_BWD, s);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(VCGS_E_HIP, std::string("kernel launch failed: ") + hipGetErrorString(e));
    return VCGS_OK;
}

int vcgs_l1_loss(vcgs_ctx* ctx, const vcgs_images* img, const float* target_color, const float* target_depth,
                 int32_t width, int32_t height, float w_depth, float* dl_dcolor, float* dl_ddepth, float* loss,
                 void* stream)
{
    if (!ctx || !img || !img->color || !img->depth || !target_color || !target_depth || !dl_dcolor || !dl_ddepth)
        return fail(VCGS_E_INVALID, "NULL argument");
    if (width <= 0 || height <= 0) return fail(VCGS_E_INVALID, "bad image size");
    HIP_TRY(hipSetDevice(ctx->device));
    const int64_t npix = (int64_t)width * height;
    Scratch sc(&ctx->pool);
    float* partial = loss ? sc.get<float>(l1_loss_blocks(npix)) : nullptr;
    if (sc.oom) return fail(VCGS_E_NOMEM, "device allocation failed (loss)");
    ctx->prof.begin(VCGS_STAGE_LOSS, (hipStream_t)stream);
    launch_l1_loss(npix, img->color, img->depth, target_color, target_depth, w_depth, dl_dcolor, dl_ddepth, loss,
                   partial, (hipStream_t)stream);
    ctx->prof.end(VCGS_STAGE_LOSS, (hipStream_t)stream);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(VCGS_E_HIP, std::string("kernel launch failed: ") + hipGetErrorString(e));
    return VCGS_OK;
}

static int make_decode_args(const vcgs_anchors* a, const vcgs_mlp* mlp, const vcgs_codebook* cb,
                            const float* mask_logit, float mask_eps, DecodeArgs* d)
{
    if (!a || !mlp) return fail(VCGS_E_INVALID, "anchors or mlp is NULL");
    if (a->n_anchor < 0) return fail(VCGS_E_INVALID, "negative anchor count");
    if (a->feat_dim != 32) return fail(VCGS_E_UNSUPPORTED, "feat_dim must be 32");
    if (a->k < 1 || a->k > 16) return fail(VCGS_E_UNSUPPORTED, "k must be in [1, 16]");
    if (a->n_anchor * a->k >= ((int64_t)1 << 31)) return fail(VCGS_E_UNSUPPORTED, "too many Gaussians");
    if (a->n_anchor > 0 && (!a->xa || !a->feat || !a->scaling || !a->offset))
        return fail(VCGS_E_INVALID, "an anchor pointer is NULL");
    if (!mlp->W1 || !mlp->b1 || !mlp->W2 || !mlp->b2) return fail(VCGS_E_INVALID, "an MLP pointer is NULL");
    d->na = a->n_anchor;
    d->k = a->k;
    d->xa = a->xa; d->feat = a->feat; d->scaling = a->scaling; d->offset = a->offset;
    d->W1 = mlp->W1; d->b1 = mlp->b1; d->W2 = mlp->W2; d->b2 = mlp->b2;
    d->stages = 0; d->cb_size = 0; d->books = nullptr; d->idx = nullptr;
    if (cb) {
        if (cb->stages < 1 || cb->size < 1 || !cb->books || !cb->idx)
            return fail(VCGS_E_INVALID, "codebook needs stages >= 1, size >= 1 and non-NULL arrays");
        d->stages = cb->stages; d->cb_size = cb->size; d->books = cb->books; d->idx = cb->idx;
    }
    d->mask_logit = mask_logit;
    d->mask_thr = 0.0f;
    if (mask_logit) {
        if (!(mask_eps > 0.0f && mask_eps < 1.0f)) return fail(VCGS_E_INVALID, "mask_eps must be in (0, 1)");
        // sigmoid(m) > eps  <=>  m > log(eps / (1 - eps))
        d->mask_thr = (float)std::log((double)mask_eps / (1.0 - (double)mask_eps));
    }
    return VCGS_OK;
}

int vcgs_decode_anchors(vcgs_ctx* ctx, const vcgs_anchors* a, const vcgs_mlp* mlp, const vcgs_codebook* cb,
                        const float* mask_logit, float mask_eps, vcgs_gaussian_buffers* out, void* stream)
{
    if (!ctx || !out) return fail(VCGS_E_INVALID, "ctx or out is NULL");
    DecodeArgs d;
    int rc = make_decode_args(a, mlp, cb, mask_logit, mask_eps, &d);
    if (rc != VCGS_OK) return rc;
    if (d.na > 0 && (!out->mean || !out->scale || !out->quat || !out->opacity || !out->color))
        return fail(VCGS_E_INVALID, "an output pointer is NULL");
    HIP_TRY(hipSetDevice(ctx->device));
    ctx->prof.begin(VCGS_STAGE_DECODE, (hipStream_t)stream);
    launch_decode_fwd(d, *out, (hipStream_t)stream);
    ctx->prof.end(VCGS_STAGE_DECODE, (hipStream_t)stream);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(VCGS_E_HIP, std::string("kernel launch failed: ") + hipGetErrorString(e));
    return VCGS_OK;
}

int vcgs_decode_anchors_backward(vcgs_ctx* ctx, const vcgs_anchors* a, const vcgs_mlp* mlp, const vcgs_codebook* cb,
                                 const float* mask_logit, float mask_eps, const vcgs_gaussian_buffers* dG,
                                 vcgs_anchor_grads* out, void* stream)
{
    if (!ctx || !out || !dG) return fail(VCGS_E_INVALID, "ctx, dG or out is NULL");
    DecodeArgs d;
    int rc = make_decode_args(a, mlp, cb, mask_logit, mask_eps, &d);
    if (rc != VCGS_OK) return rc;
    HIP_TRY(hipSetDevice(ctx->device));
    hipStream_t s = (hipStream_t)stream;
    vcgs_anchor_grads o = *out;
    if (!cb) o.books = nullptr;
    if (!mask_logit) o.mask_logit = nullptr;
    if (d.na == 0) return VCGS_OK;
    Scratch sc(&ctx->pool);
    const int nb = decode_bwd_blocks(d.na);
    float* partial = sc.get<float>((int64_t)nb * decode_bwd_partial_floats(d.k));
    if (sc.oom) return fail(VCGS_E_NOMEM, "device allocation failed (decode backward)");
    ctx->prof.begin(VCGS_STAGE_DECODE_BWD, s);
    launch_decode_bwd(d, *dG, o, partial, nb, s);
    ctx->prof.end(VCGS_STAGE_DECODE_BWD, s);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(VCGS_E_HIP, std::string("kernel launch failed: ") + hipGetErrorString(e));
    return VCGS_OK;
}

int vcgs_set_option(int key, int value)
{
    Options& o = options();
    switch (key) {
    case VCGS_OPT_PPL_FWD:
    case VCGS_OPT_PPL_BWD:
        if (value != 1 && value != 2 && value != 4) return fail(VCGS_E_INVALID, "pixels per lane must be 1, 2 or 4");
        (key == VCGS_OPT_PPL_FWD ? o.ppl_fwd : o.ppl_bwd) = value;
        return VCGS_OK;
    case VCGS_OPT_CULL:
        if (value != 0 && value != 1) return fail(VCGS_E_INVALID, "cull must be 0 or 1");
        o.cull = value;
        return VCGS_OK;
    default:
        return fail(VCGS_E_INVALID, "unknown option");
    }
}

int vcgs_get_option(int key, int* value)
{
    if (!value) return fail(VCGS_E_INVALID, "value is NULL");
    const Options& o = options();
    switch (key) {
    case VCGS_OPT_PPL_FWD: *value = o.ppl_fwd; return VCGS_OK;
    case VCGS_OPT_PPL_BWD: *value = o.ppl_bwd; return VCGS_OK;
    case VCGS_OPT_CULL: *value = o.cull; return VCGS_OK;
    default: return fail(VCGS_E_INVALID, "unknown option");
    }
}

int vcgs_profile_enable(vcgs_ctx* ctx, int on)
{
    if (!ctx) return fail(VCGS_E_INVALID, "ctx is NULL");
    HIP_TRY(hipSetDevice(ctx->device));
    ctx->prof.clear();
    ctx->prof.on = on != 0;
    return VCGS_OK;
}

int vcgs_profile_read(vcgs_ctx* ctx, int stage, double* total_ms, int64_t* launches)
{
    if (!ctx || stage < 0 || stage >= VCGS_STAGE_COUNT) return fail(VCGS_E_INVALID, "bad ctx or stage");
    HIP_TRY(hipSetDevice(ctx->device));
    ctx->prof.fold();
    if (total_ms) *total_ms = ctx->prof.ms[stage];
    if (launches) *launches = ctx->prof.launches[stage];
    return VCGS_OK;
}

int vcgs_count_enable(vcgs_ctx* ctx, int on)
{
    if (!ctx) return fail(VCGS_E_INVALID, "ctx is NULL");
    HIP_TRY(hipSetDevice(ctx->device));
    if (on && !ctx->prof.d_counters) {
        HIP_TRY(hipMalloc((void**)&ctx->prof.d_counters, 8 * sizeof(unsigned long long)));
        HIP_TRY(hipMemset(ctx->prof.d_counters, 0, 8 * sizeof(unsigned long long)));
    }
    ctx->prof.count = on != 0;
    return VCGS_OK;
}

int vcgs_count_read(vcgs_ctx* ctx, int64_t out[5])
{
    if (!ctx || !out) return fail(VCGS_E_INVALID, "NULL argument");
    if (!ctx->prof.d_counters) {
        for (int i = 0; i < 5; ++i) out[i] = 0;
        return VCGS_OK;
    }
    HIP_TRY(hipSetDevice(ctx->device));
    unsigned long long h[5];
    HIP_TRY(hipDeviceSynchronize());
    HIP_TRY(hipMemcpy(h, ctx->prof.d_counters, sizeof(h), hipMemcpyDeviceToHost));
    for (int i = 0; i < 5; ++i) out[i] = (int64_t)h[i];
    return VCGS_OK;
}

}  // extern "C"
