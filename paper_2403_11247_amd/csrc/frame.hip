// Render orchestration: one core that renders n_views views of the same
// Gaussians (forward, then optionally the replayed backward), used by
//   - vcgs_render_forward / vcgs_render_backward: one view, buffers from the
//     context pool, one stream synchronisation to size the pair buffers;
//   - vcgs_render_batch: up to 16 views in one pass (bundle-adjustment window
//     or a serving step), buffers owned by a prepared plan whose pair capacity
//     is sized once; with VCGS_BATCH_GRAPH the whole pass -- projection, sorts,
//     compositing, loss, backward -- is captured once into a hipGraph and then
//     replayed as a single launch, with the poses read from device memory.
//
// Entry e of the per-Gaussian arrays is (view e / n, Gaussian e % n); global
// tile ids are view-major, so the depth sort over all entries followed by the
// stable tile sort gives every tile of every view its own depth-ordered list.
#include <cmath>

#include "frame.h"

using namespace vcgs;

namespace vcgs {

void build_tables(int V, int64_t n, const vcgs_camera* cams, const vcgs_pose* poses, const float bg[3],
                         Frame& f)
{
    f.V = V;
    f.n = n;
    f.E = n * V;
    std::memset(&f.pt, 0, sizeof(f.pt));
    std::memset(&f.et, 0, sizeof(f.et));
    std::memset(&f.vt, 0, sizeof(f.vt));
    uint32_t base = 0;
    for (int i = 0; i < V; ++i) {
        const CamK c = make_camk(cams[i], base);
        f.pt.cam[i] = c;
        f.pt.pose[i] = make_posek(poses[i]);
        f.et.tiles_x[i] = c.tiles_x;
        f.et.tile_base[i] = base;
        f.vt.cam[i] = c;
        base += (uint32_t)(c.tiles_x * c.tiles_y);
        f.vt.tile_end[i] = base;
    }
    f.pt.n_views = f.et.n_views = f.vt.n_views = V;
    f.pt.n = f.et.n = f.vt.n = n;
    f.total_tiles = base;
    for (int i = 0; i < 3; ++i) f.vt.bg[i] = bg[i];
}

// What a pass needs at zero: both sorts' counters, the tile ranges, the pair
// scan's look-back words and (unless keep_overflow) the overflow flag.
static ZeroSegs pass_zero_segs(Frame& f, Work& w, bool keep_overflow)
{
    ZeroSegs z{};
    z.p[0] = w.headE;
    z.n[0] = sort_head_words();
    z.p[1] = w.headP;
    z.n[1] = sort_head_words();
    z.p[2] = f.ranges;
    z.n[2] = 2 * (int64_t)f.total_tiles;
    z.p[3] = keep_overflow ? nullptr : w.overflow;
    z.n[3] = 1;
    z.p[4] = w.scanE;
    z.n[4] = pair_scan_words(f.E);
    return z;
}

void zero_pass(Frame& f, Work& w, hipStream_t s, bool keep_overflow)
{
    launch_zero_u32(pass_zero_segs(f, w, keep_overflow), s);
}

// Projection, depth order of all entries, pair offsets; the pair count ends
// up in w.total on the device.  Returns the depth order.
const uint32_t* phase_a(Prof& pf, const vcgs_gaussians& g, Frame& f, Work& w, hipStream_t s, bool keep_overflow,
                        uint32_t* host_total)
{
    // the projection's threads also clear what zero_pass would (one launch fewer)
    const ZeroSegs z = pass_zero_segs(f, w, keep_overflow);
    pf.begin(VCGS_STAGE_PREPROCESS, s);
    launch_preprocess(f.pt, f.pt_dev, g, f.rec, f.depth_key, f.rect, f.count, f.g2, s, &z, f.tab_by_value);
    pf.end(VCGS_STAGE_PREPROCESS, s);
    pf.begin(VCGS_STAGE_DEPTH_SORT, s);
    // culled entries carry the drop key and leave the depth order in its first pass
    const SortTemp t{w.kaltE, w.valtE, w.headE, w.stateE};
    const int which = radix_sort_u32(w.dk, w.order, true, Count{f.E, nullptr}, 32, t, s, &w.nvis, f.depth_key);
    pf.end(VCGS_STAGE_DEPTH_SORT, s);
    const uint32_t* ord = which ? w.valtE : w.order;
    pf.begin(VCGS_STAGE_PAIR_SCAN, s);
    pair_offsets(ord, f.count, Count{f.E, w.nvis}, w.cnt, w.offs, w.total, w.scanE, s, host_total);
    pf.end(VCGS_STAGE_PAIR_SCAN, s);
    return ord;
}

// Pairs, stable tile sort, tile ranges, forward compositing.
void phase_b(Prof& pf, Frame& f, Work& w, const uint32_t* ord, hipStream_t s)
{
    if (f.cap > 0) {
        const Count P{f.cap, w.total};
        const int end_bit = bits_for(f.total_tiles - 1);
        const SortTemp tp{w.kaltP, w.valtP, w.headP, w.stateP, w.stateP_words};
        // the emission builds the tile sort's histograms (the projection launch cleared them)
        const SortPrep sp = radix_sort_prep(P, end_bit, tp, f.pair_hint);
        pf.begin(VCGS_STAGE_EMIT, s);
        // grids follow the expected count (with a margin) when the capacity is only a bound
        const int64_t grid_items =
            f.pair_hint > 0 ? std::min<int64_t>(f.cap, f.pair_hint + f.pair_hint / 2 + 4096) : f.cap;
        const bool hist = launch_emit_pairs(f.et, f.E, w.nvis, ord, w.offs, w.cnt, f.rect, w.scanP, w.tile_ids,
                                            f.gids, f.cap, w.total, w.overflow, sp, s, grid_items) &&
                          sp.ghist != nullptr;
        pf.end(VCGS_STAGE_EMIT, s);
        pf.begin(VCGS_STAGE_TILE_SORT, s);
        const int ws = radix_sort_u32(w.tile_ids, f.gids, false, P, end_bit, tp, s, nullptr, nullptr, f.pair_hint,
                                      hist);
        const uint32_t* tsorted = ws ? w.kaltP : w.tile_ids;
        if (ws) launch_copy_u32(f.gids, w.valtP, P, s);
        pf.end(VCGS_STAGE_TILE_SORT, s);
        pf.begin(VCGS_STAGE_TILE_RANGES, s);
        launch_tile_ranges(P, tsorted, f.total_tiles, f.ranges, s, grid_items);
        pf.end(VCGS_STAGE_TILE_RANGES, s);
    }
    unsigned long long* cnts = nullptr;
    if (pf.count && pf.d_counters && !pf.capturing) {
        cnts = pf.d_counters;
        launch_fill_u32(reinterpret_cast<uint32_t*>(cnts), 0u, 4, s);
    }
    pf.begin(VCGS_STAGE_COMPOSITE, s);
    launch_composite_fwd(f.vt, f.total_tiles, f.rec, f.gids, f.ranges, cnts, s);
    pf.end(VCGS_STAGE_COMPOSITE, s);
}

// Replayed compositing adjoint and projection adjoint; g2 holds 12 floats per
// entry (zero on entry for every visible one: the forward's projection zeroes
// them when the frame's g2 is set, else fill_g2 does), partial 6 floats per
// (view, block).
static void backward_core(vcgs_ctx* ctx, Frame& f, const vcgs_gaussians& g, const vcgs_gaussian_buffers& gb,
                          float* dl_dpose, float* g2, float* partial, int pb, hipStream_t s, bool fill_g2)
{
    Prof& pf = ctx->prof;
    unsigned long long* cnts = nullptr;
    if (pf.count && pf.d_counters && !pf.capturing) {
        cnts = pf.d_counters;
        launch_fill_u32(reinterpret_cast<uint32_t*>(cnts) + 4, 0u, 6, s);
    }
    if (fill_g2) launch_fill_f32(g2, 0.0f, (int64_t)kG2 * f.E, s);
    pf.begin(VCGS_STAGE_COMPOSITE_BWD, s);
    if (f.cap > 0) launch_composite_bwd(f.vt, f.total_tiles, f.rec, f.gids, f.ranges, g2, cnts, s);
    pf.end(VCGS_STAGE_COMPOSITE_BWD, s);
    pf.begin(VCGS_STAGE_PREPROCESS_BWD, s);
    if (f.n > 0) launch_preprocess_bwd(f.pt, f.pt_dev, g, f.count, f.rec, g2, gb, partial, pb, s);
    else launch_fill_f32(partial, 0.0f, 6 * (int64_t)f.V, s);
    if (dl_dpose) launch_pose_reduce(partial, f.V, f.n > 0 ? pb : 1, dl_dpose, s);
    pf.end(VCGS_STAGE_PREPROCESS_BWD, s);
}

int check_camera(const vcgs_camera* c)
{
    if (!c) return fail(VCGS_E_INVALID, "camera is NULL");
    if (c->width <= 0 || c->height <= 0) return fail(VCGS_E_INVALID, "camera width/height must be positive");
    if (c->width > 65535 * kTile || c->height > 65535 * kTile) return fail(VCGS_E_UNSUPPORTED, "image too large");
    if (c->tile != kTile) return fail(VCGS_E_INVALID, "camera tile must be 16");
    if (!(c->fx > 0.0f) || !(c->fy > 0.0f)) return fail(VCGS_E_INVALID, "focal lengths must be positive");
    return VCGS_OK;
}

int check_gaussians(const vcgs_gaussians* g, int V)
{
    if (!g) return fail(VCGS_E_INVALID, "gaussians is NULL");
    if (g->n < 0) return fail(VCGS_E_INVALID, "negative Gaussian count");
    if (g->n * std::max(V, 1) > kMaxSortItems) return fail(VCGS_E_UNSUPPORTED, "at most 2^30-1 Gaussian-view entries");
    if (g->n > 0 && (!g->mean || !g->scale || !g->quat || !g->opacity || !g->color))
        return fail(VCGS_E_INVALID, "a Gaussian attribute pointer is NULL");
    return VCGS_OK;
}

// ---------------------------------------------------------------------------
// Batched plans
// ---------------------------------------------------------------------------
struct BatchPlan {
    // signature
    int64_t n = 0;
    int V = 0;
    int flags = 0;
    bool backward = false;
    vcgs_camera cams[kMaxViews];
    std::vector<const void*> ptrs;
    float bg[3];
    float w_depth = 0.5f;
    // buffers
    Frame f;
    Work w{};
    float* dlc[kMaxViews] = {};
    float* dld[kMaxViews] = {};
    float* loss_partial = nullptr;
    int loss_blocks = 0;
    float* g2 = nullptr;
    float* partial = nullptr;
    int pb = 0;
    bool graph_g2 = false;   // the captured forward zeroes g2 (f.g2 was set at capture)
    bool g2_zeroed = false;  // the last forward zeroed g2 and no backward has used it since
    // pinned staging of the per-view table, two slots used in turn: a pass
    // only waits for the upload of the pass before the previous one
    ProjTab* pt_host[2] = {};
    uint32_t* host_flags = nullptr;  // pinned: pair count, overflow
    hipEvent_t tab_copied[2] = {};
    bool tab_pending[2] = {};
    int tab_slot = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    // a forward kept for the caller's backward (vcgs_render_batch_forward):
    // the backward's own captured graph and the pointers it was captured with
    bool split = false;
    hipGraph_t graph_bwd = nullptr;
    hipGraphExec_t exec_bwd = nullptr;
    std::vector<const void*> bwd_ptrs;
    std::vector<void*> blocks_e, blocks_p;
    int64_t need = 0;
    vcgs_ctx* ctx = nullptr;

    template <class T>
    T* get_e(int64_t c)
    {
        void* p = ctx->pool.alloc((size_t)std::max<int64_t>(c, 1) * sizeof(T));
        blocks_e.push_back(p);
        return static_cast<T*>(p);
    }
    template <class T>
    T* get_p(int64_t c)
    {
        void* p = ctx->pool.alloc((size_t)std::max<int64_t>(c, 1) * sizeof(T));
        blocks_p.push_back(p);
        return static_cast<T*>(p);
    }
    bool ok() const
    {
        for (void* b : blocks_e)
            if (!b) return false;
        for (void* b : blocks_p)
            if (!b) return false;
        return true;
    }
    void drop_graph()
    {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        if (exec_bwd) (void)hipGraphExecDestroy(exec_bwd);
        if (graph_bwd) (void)hipGraphDestroy(graph_bwd);
        exec = nullptr;
        graph = nullptr;
        exec_bwd = nullptr;
        graph_bwd = nullptr;
        bwd_ptrs.clear();
    }
    void release_p()
    {
        for (void* b : blocks_p) ctx->pool.free(b);
        blocks_p.clear();
    }
    void release()
    {
        drop_graph();
        release_p();
        for (void* b : blocks_e) ctx->pool.free(b);
        blocks_e.clear();
        for (int i = 0; i < 2; ++i) {
            if (pt_host[i]) (void)hipHostFree(pt_host[i]);
            if (tab_copied[i]) (void)hipEventDestroy(tab_copied[i]);
            pt_host[i] = nullptr;
            tab_copied[i] = nullptr;
            tab_pending[i] = false;
        }
        if (host_flags) (void)hipHostFree(host_flags);
        host_flags = nullptr;
    }
};

void destroy_plans(vcgs_ctx* ctx)
{
    (void)hipDeviceSynchronize();
    for (BatchPlan* p : ctx->plans) {
        p->release();
        delete p;
    }
    ctx->plans.clear();
    ctx->last_plan = nullptr;
    ctx->fwd_plan = nullptr;
    if (ctx->graph_stream) (void)hipStreamDestroy(ctx->graph_stream);
    ctx->graph_stream = nullptr;
}

// Everything one pass of a plan enqueues (also what a graph captures).
static void enqueue_plan(vcgs_ctx* ctx, BatchPlan& p, const vcgs_gaussians& g, const vcgs_images* outs,
                         const float* const* tc, const float* const* td, const vcgs_gaussian_buffers& gb,
                         float* dl_dpose, float* loss, hipStream_t s)
{
    const uint32_t* ord = phase_a(ctx->prof, g, p.f, p.w, s, true);
    phase_b(ctx->prof, p.f, p.w, ord, s);
    if (!p.backward) return;
    ctx->prof.begin(VCGS_STAGE_LOSS, s);
    LossTab lt;
    std::memset(&lt, 0, sizeof(lt));
    lt.n_views = p.V;
    lt.w_depth = p.w_depth;
    for (int v = 0; v < p.V; ++v) {
        lt.npix[v] = (int64_t)p.cams[v].width * p.cams[v].height;
        lt.block0[v + 1] = lt.block0[v] + l1_loss_blocks(lt.npix[v]);
        lt.c[v] = outs[v].color;
        lt.d[v] = outs[v].depth;
        lt.tc[v] = tc[v];
        lt.td[v] = td[v];
        lt.dlc[v] = p.dlc[v];
        lt.dld[v] = p.dld[v];
    }
    launch_l1_loss_views(lt, loss, p.loss_partial, s);
    ctx->prof.end(VCGS_STAGE_LOSS, s);
    // the pass's projection zeroed the gradient slots (the plan's frame carries g2)
    backward_core(ctx, p.f, g, gb, dl_dpose, p.g2, p.partial, p.pb, s, false);
}

}  // namespace vcgs

// Saved forward of one view.
struct vcgs_state {
    vcgs_ctx* ctx = nullptr;
    Frame f;
    int64_t P = 0;
    float* t_final = nullptr;
    uint32_t* n_contrib = nullptr;
    bool g2_clean = false;  // f.g2 zeroed by the forward and not used by a backward since
    std::vector<void*> blocks;

    template <class T>
    T* get(int64_t c)
    {
        void* p = ctx->pool.alloc((size_t)std::max<int64_t>(c, 1) * sizeof(T));
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

extern "C" {

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
    out->n = st->f.n;
    out->n_pairs = st->P;
    out->tiles_x = st->f.pt.cam[0].tiles_x;
    out->tiles_y = st->f.pt.cam[0].tiles_y;
    out->depth_bits = st->f.depth_key;
    out->rect = reinterpret_cast<const uint16_t*>(st->f.rect);
    out->count = st->f.count;
    out->gids = st->f.gids;
    out->ranges = st->f.ranges;
    out->t_final = st->t_final;
    out->n_contrib = st->n_contrib;
    out->splats = reinterpret_cast<const float*>(st->f.rec);
    return VCGS_OK;
}

static int render_forward_impl(vcgs_ctx* ctx, const vcgs_gaussians* g, const vcgs_camera* cam,
                               const vcgs_pose* pose, const float bg[3], vcgs_images* out, vcgs_state** state_out,
                               uint32_t* hits, void* stream)
{
    if (!ctx) return fail(VCGS_E_INVALID, "ctx is NULL");
    int rc;
    if ((rc = check_gaussians(g, 1)) != VCGS_OK) return rc;
    if ((rc = check_camera(cam)) != VCGS_OK) return rc;
    if (!pose || !bg || !out || !out->color || !out->depth || !out->alpha)
        return fail(VCGS_E_INVALID, "pose, bg or an output image is NULL");
    if (state_out) *state_out = nullptr;
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(hipSetDevice(ctx->device));

    vcgs_state* st = new vcgs_state();
    st->ctx = ctx;
    Frame& f = st->f;
    build_tables(1, g->n, cam, pose, bg, f);
    const int64_t HW = (int64_t)cam->width * cam->height;
    f.pt_dev = st->get<ProjTab>(1);
    f.rec = st->get<Splat>(f.E);
    f.depth_key = st->get<uint32_t>(f.E);
    f.rect = st->get<uint2>(f.E);
    f.count = st->get<uint32_t>(f.E);
    f.ranges = st->get<uint32_t>(2 * (int64_t)f.total_tiles);
    st->t_final = st->get<float>(HW);
    st->n_contrib = st->get<uint32_t>(HW);
    // a kept state carries the backward's gradient slots, zeroed by the projection
    if (state_out) f.g2 = st->get<float>((int64_t)kG2 * f.E);
    f.vt.color[0] = out->color;
    f.vt.depth[0] = out->depth;
    f.vt.alpha[0] = out->alpha;
    f.vt.t_final[0] = st->t_final;
    f.vt.n_contrib[0] = st->n_contrib;
    f.vt.hits = hits;
    auto drop = [&](int code, const std::string& m) {
        st->release();
        delete st;
        return fail(code, m);
    };
    if (!st->ok()) return drop(VCGS_E_NOMEM, "device allocation failed (state)");
    {
        Scratch sc(&ctx->pool);
        Work w{};
        alloc_work_e(w, f.E, [&](int64_t c) { return sc.get<uint32_t>(c); });
        if (sc.oom) return drop(VCGS_E_NOMEM, "device allocation failed (depth sort)");
        // the projection takes the table as a kernel argument and leaves the
        // device copy the backward reads; with nothing to project it is
        // uploaded (the stream is synchronised below, so the pinned staging
        // copy is free again on return)
        f.tab_by_value = f.E > 0;
        if (!f.tab_by_value) {
            std::memcpy(ctx->host_tab, &f.pt, sizeof(ProjTab));
            if (hipMemcpyAsync(f.pt_dev, ctx->host_tab, sizeof(ProjTab), hipMemcpyHostToDevice, s) != hipSuccess)
                return drop(VCGS_E_HIP, "table upload failed");
        }
        const uint32_t* ord = nullptr;
        // the pair scan also writes the pair count into the pinned word: no copy before the synchronisation
        if (f.E > 0) ord = phase_a(ctx->prof, *g, f, w, s, false, ctx->host_u32);
        else zero_pass(f, w, s);
        if (f.E > 0) {
            if (hipStreamSynchronize(s) != hipSuccess)
                return drop(VCGS_E_HIP, std::string("pair count readback failed: ") +
                                            hipGetErrorString(hipGetLastError()));
            st->P = ctx->host_u32[0];
            if (st->P > kMaxSortItems) return drop(VCGS_E_UNSUPPORTED, "more than 2^30-1 (tile, Gaussian) pairs");
        }
        f.cap = st->P;
        f.gids = st->get<uint32_t>(f.cap);
        if (f.cap > 0) alloc_work_p(w, f.cap, [&](int64_t c) { return sc.get<uint32_t>(c); });
        if (!st->ok() || sc.oom) return drop(VCGS_E_NOMEM, "device allocation failed (pairs)");
        phase_b(ctx->prof, f, w, ord, s);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return drop(VCGS_E_HIP, std::string("kernel launch failed: ") + hipGetErrorString(e));
    }
    if (state_out) {
        st->g2_clean = f.g2 != nullptr;
        *state_out = st;
    } else {
        st->release();
        delete st;
    }
    return VCGS_OK;
}

int vcgs_render_forward(vcgs_ctx* ctx, const vcgs_gaussians* g, const vcgs_camera* cam, const vcgs_pose* pose,
                        const float bg[3], vcgs_images* out, vcgs_state** state_out, void* stream)
{
    return render_forward_impl(ctx, g, cam, pose, bg, out, state_out, nullptr, stream);
}

int vcgs_render_forward_hits(vcgs_ctx* ctx, const vcgs_gaussians* g, const vcgs_camera* cam, const vcgs_pose* pose,
                             const float bg[3], vcgs_images* out, vcgs_state** state_out, uint32_t* hits,
                             void* stream)
{
    if (!hits) return fail(VCGS_E_INVALID, "hits is NULL");
    return render_forward_impl(ctx, g, cam, pose, bg, out, state_out, hits, stream);
}

int vcgs_render_backward(vcgs_ctx* ctx, const vcgs_state* st_, const vcgs_gaussians* g, const vcgs_camera* cam,
                         const vcgs_pose* pose, const float* dl_dcolor, const float* dl_ddepth,
                         const float* dl_dalpha, vcgs_gaussian_buffers* grads, float* dl_dpose, void* stream)
{
    if (!ctx || !st_) return fail(VCGS_E_INVALID, "ctx or state is NULL");
    int rc;
    if ((rc = check_gaussians(g, 1)) != VCGS_OK) return rc;
    if ((rc = check_camera(cam)) != VCGS_OK) return rc;
    if (!pose) return fail(VCGS_E_INVALID, "pose is NULL");
    vcgs_state* st = const_cast<vcgs_state*>(st_);
    if (g->n != st->f.n || cam->width != st->f.pt.cam[0].W || cam->height != st->f.pt.cam[0].H)
        return fail(VCGS_E_INVALID, "Gaussians or camera differ from the forward call");
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(hipSetDevice(ctx->device));
    const vcgs_gaussian_buffers gb =
        grads ? *grads : vcgs_gaussian_buffers{nullptr, nullptr, nullptr, nullptr, nullptr};
    Frame f = st->f;  // the saved tables with this call's upstream gradients
    f.vt.dl_dc[0] = dl_dcolor;
    f.vt.dl_dd[0] = dl_ddepth;
    f.vt.dl_da[0] = dl_dalpha;
    Scratch sc(&ctx->pool);
    const int pb = std::max(1, preprocess_bwd_blocks(f.n));
    float* partial = sc.get<float>(6 * (int64_t)pb * f.V);
    if (sc.oom || !st->f.g2) return fail(VCGS_E_NOMEM, "device allocation failed (backward)");
    // a second backward of the same state starts from zero again
    backward_core(ctx, f, *g, gb, dl_dpose, st->f.g2, partial, pb, s, !st->g2_clean);
    st->g2_clean = false;
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(VCGS_E_HIP, std::string("kernel launch failed: ") + hipGetErrorString(e));
    return VCGS_OK;
}

// split: a forward only, kept for a later vcgs_render_batch_backward.
static int render_batch_impl(vcgs_ctx* ctx, const vcgs_gaussians* g, const vcgs_views* views, const float bg[3],
                             const float* const* target_color, const float* const* target_depth, float w_depth,
                             const vcgs_images* outs, vcgs_gaussian_buffers* grads, float* dl_dpose, float* loss,
                             int flags, uint32_t* hits, bool split, void* stream)
{
    if (!ctx || !views || !outs || !bg) return fail(VCGS_E_INVALID, "ctx, views, outs or bg is NULL");
    const int V = views->n_views;
    if (V < 1 || V > kMaxViews) return fail(VCGS_E_UNSUPPORTED, "n_views must be in [1, 16]");
    if (!views->cams || !views->poses) return fail(VCGS_E_INVALID, "cams or poses is NULL");
    int rc;
    if ((rc = check_gaussians(g, V)) != VCGS_OK) return rc;
    for (int v = 0; v < V; ++v) {
        if ((rc = check_camera(&views->cams[v])) != VCGS_OK) return rc;
        if (!outs[v].color || !outs[v].depth || !outs[v].alpha) return fail(VCGS_E_INVALID, "an output image is NULL");
    }
    const bool backward = grads != nullptr || dl_dpose != nullptr;
    if (backward && (!target_color || !target_depth))
        return fail(VCGS_E_INVALID, "the backward needs target images");
    if (backward)
        for (int v = 0; v < V; ++v)
            if (!target_color[v] || !target_depth[v]) return fail(VCGS_E_INVALID, "a target image is NULL");
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(hipSetDevice(ctx->device));
    const vcgs_gaussian_buffers gb =
        grads ? *grads : vcgs_gaussian_buffers{nullptr, nullptr, nullptr, nullptr, nullptr};

    // signature of the prepared plan: shapes, intrinsics and every pointer a graph would bake in
    std::vector<const void*> ptrs = {g->mean, g->scale, g->quat, g->opacity, g->color, gb.mean, gb.scale, gb.quat,
                                     gb.opacity, gb.color, dl_dpose, loss, hits};
    for (int v = 0; v < V; ++v) {
        ptrs.push_back(outs[v].color);
        ptrs.push_back(outs[v].depth);
        ptrs.push_back(outs[v].alpha);
        ptrs.push_back(backward ? target_color[v] : nullptr);
        ptrs.push_back(backward ? target_depth[v] : nullptr);
    }
    BatchPlan* plan = nullptr;
    for (BatchPlan* p : ctx->plans) {
        bool same = p->n == g->n && p->V == V && p->flags == flags && p->backward == backward &&
                    p->split == split && p->ptrs == ptrs && p->w_depth == w_depth &&
                    std::memcmp(p->bg, bg, sizeof(p->bg)) == 0;
        for (int v = 0; same && v < V; ++v) same = std::memcmp(&p->cams[v], &views->cams[v], sizeof(vcgs_camera)) == 0;
        if (same) {
            plan = p;
            break;
        }
    }
    if (!plan) {
        if (ctx->plans.size() >= 32) {  // keep a few plans; drop the oldest
            BatchPlan* old = ctx->plans.front();
            (void)hipDeviceSynchronize();  // its last pass may have run on another stream
            if (ctx->last_plan == old) ctx->last_plan = nullptr;
            if (ctx->fwd_plan == old) ctx->fwd_plan = nullptr;
            old->release();
            delete old;
            ctx->plans.erase(ctx->plans.begin());
        }
        plan = new BatchPlan();
        plan->ctx = ctx;
        plan->n = g->n;
        plan->V = V;
        plan->flags = flags;
        plan->backward = backward;
        plan->split = split;
        plan->ptrs = ptrs;
        plan->w_depth = w_depth;
        for (int i = 0; i < 3; ++i) plan->bg[i] = bg[i];
        for (int v = 0; v < V; ++v) plan->cams[v] = views->cams[v];
        Frame& f = plan->f;
        build_tables(V, g->n, views->cams, views->poses, bg, f);
        f.pt.per_view = (flags & VCGS_BATCH_PER_VIEW) ? 1 : 0;
        f.vt.hits = hits;
        f.pt_dev = plan->get_e<ProjTab>(1);
        f.rec = plan->get_e<Splat>(f.E);
        f.depth_key = plan->get_e<uint32_t>(f.E);
        f.rect = plan->get_e<uint2>(f.E);
        f.count = plan->get_e<uint32_t>(f.E);
        f.ranges = plan->get_e<uint32_t>(2 * (int64_t)f.total_tiles);
        int64_t max_pix = 0;
        for (int v = 0; v < V; ++v) {
            const int64_t HW = (int64_t)views->cams[v].width * views->cams[v].height;
            max_pix = std::max(max_pix, HW);
            f.vt.color[v] = outs[v].color;
            f.vt.depth[v] = outs[v].depth;
            f.vt.alpha[v] = outs[v].alpha;
            f.vt.t_final[v] = plan->get_e<float>(HW);
            f.vt.n_contrib[v] = plan->get_e<uint32_t>(HW);
            if (backward) {
                plan->dlc[v] = plan->get_e<float>(3 * HW);
                plan->dld[v] = plan->get_e<float>(HW);
                f.vt.dl_dc[v] = plan->dlc[v];
                f.vt.dl_dd[v] = plan->dld[v];
            }
        }
        alloc_work_e(plan->w, f.E, [&](int64_t c) { return plan->get_e<uint32_t>(c); });
        if (backward) {
            plan->loss_blocks = l1_loss_blocks(max_pix);
            plan->loss_partial = plan->get_e<float>((int64_t)V * plan->loss_blocks);
            plan->pb = std::max(1, preprocess_bwd_blocks(f.n));
            plan->g2 = plan->get_e<float>((int64_t)kG2 * f.E);
            f.g2 = plan->g2;  // every pass's projection zeroes the gradient slots
            plan->partial = plan->get_e<float>(6 * (int64_t)plan->pb * V);
        }
        bool ok = plan->ok() && hipHostMalloc((void**)&plan->host_flags, 16, hipHostMallocDefault) == hipSuccess;
        for (int i = 0; ok && i < 2; ++i)
            ok = hipHostMalloc((void**)&plan->pt_host[i], sizeof(ProjTab), hipHostMallocDefault) == hipSuccess &&
                 hipEventCreateWithFlags(&plan->tab_copied[i], hipEventDisableTiming) == hipSuccess;
        if (!ok) {
            plan->release();
            delete plan;
            return fail(VCGS_E_NOMEM, "allocation failed (batch plan)");
        }
        launch_fill_u32(plan->w.overflow, 0u, 1, s);  // cleared again by each vcgs_batch_check
        ctx->plans.push_back(plan);
    }
    Frame& f = plan->f;
    // poses of this call, staged through pinned memory into the device table
    const int slot = plan->tab_slot;
    plan->tab_slot ^= 1;
    if (plan->tab_pending[slot]) HIP_TRY(hipEventSynchronize(plan->tab_copied[slot]));
    for (int v = 0; v < V; ++v) f.pt.pose[v] = make_posek(views->poses[v]);
    std::memcpy(plan->pt_host[slot], &f.pt, sizeof(ProjTab));
    HIP_TRY(hipMemcpyAsync(f.pt_dev, plan->pt_host[slot], sizeof(ProjTab), hipMemcpyHostToDevice, s));
    HIP_TRY(hipEventRecord(plan->tab_copied[slot], s));
    plan->tab_pending[slot] = true;

    // size the pair buffers once (and again after an overflow was reported)
    if (f.cap == 0 || plan->need > f.cap) {
        plan->drop_graph();
        const uint32_t* ord = phase_a(ctx->prof, *g, f, plan->w, s, true);
        (void)ord;
        HIP_TRY(hipMemcpyAsync(plan->host_flags, plan->w.total, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        const int64_t P = std::max<int64_t>(plan->host_flags[0], plan->need);
        if (P > kMaxSortItems) return fail(VCGS_E_UNSUPPORTED, "more than 2^30-1 (tile, Gaussian) pairs");
        plan->release_p();
        f.cap = std::min<int64_t>(std::max<int64_t>(P + P / 8 + 4096, 4096), kMaxSortItems);
        f.gids = plan->get_p<uint32_t>(f.cap);
        alloc_work_p(plan->w, f.cap, [&](int64_t c) { return plan->get_p<uint32_t>(c); });
        if (!plan->ok()) return fail(VCGS_E_NOMEM, "allocation failed (batch pairs)");
    }

    if (flags & VCGS_BATCH_GRAPH) {
        if (!ctx->graph_stream) HIP_TRY(hipStreamCreateWithFlags(&ctx->graph_stream, hipStreamNonBlocking));
        hipStream_t gs = ctx->graph_stream;
        if (!plan->exec) {
            // capture on the library's own stream (the caller's may be the null stream)
            HIP_TRY(hipStreamSynchronize(s));
            ctx->prof.capturing = true;
            hipError_t e = hipStreamBeginCapture(gs, hipStreamCaptureModeThreadLocal);
            if (e == hipSuccess) {
                enqueue_plan(ctx, *plan, *g, outs, target_color, target_depth, gb, dl_dpose, loss, gs);
                e = hipStreamEndCapture(gs, &plan->graph);
            }
            ctx->prof.capturing = false;
            if (e != hipSuccess) {
                plan->drop_graph();
                return fail(VCGS_E_HIP, std::string("graph capture failed: ") + hipGetErrorString(e));
            }
            HIP_TRY(hipGraphInstantiate(&plan->exec, plan->graph, nullptr, nullptr, 0));
            plan->graph_g2 = f.g2 != nullptr;
        }
        // captured on the library's stream, replayed in order on the caller's
        HIP_TRY(hipGraphLaunch(plan->exec, s));
    } else {
        enqueue_plan(ctx, *plan, *g, outs, target_color, target_depth, gb, dl_dpose, loss, s);
    }
    ctx->last_plan = plan;
    ctx->last_stream = s;
    plan->g2_zeroed = (flags & VCGS_BATCH_GRAPH) ? plan->graph_g2 : f.g2 != nullptr;
    if (split) ctx->fwd_plan = plan;
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(VCGS_E_HIP, std::string("kernel launch failed: ") + hipGetErrorString(e));
    return VCGS_OK;
}

int vcgs_render_batch(vcgs_ctx* ctx, const vcgs_gaussians* g, const vcgs_views* views, const float bg[3],
                      const float* const* target_color, const float* const* target_depth, float w_depth,
                      const vcgs_images* outs, vcgs_gaussian_buffers* grads, float* dl_dpose, float* loss,
                      int flags, void* stream)
{
    return render_batch_impl(ctx, g, views, bg, target_color, target_depth, w_depth, outs, grads, dl_dpose, loss,
                             flags, nullptr, false, stream);
}

int vcgs_render_batch_hits(vcgs_ctx* ctx, const vcgs_gaussians* g, const vcgs_views* views, const float bg[3],
                           const float* const* target_color, const float* const* target_depth, float w_depth,
                           const vcgs_images* outs, vcgs_gaussian_buffers* grads, float* dl_dpose, float* loss,
                           int flags, uint32_t* hits, void* stream)
{
    if (!hits) return fail(VCGS_E_INVALID, "hits is NULL");
    return render_batch_impl(ctx, g, views, bg, target_color, target_depth, w_depth, outs, grads, dl_dpose, loss,
                             flags, hits, false, stream);
}

int vcgs_render_batch_forward(vcgs_ctx* ctx, const vcgs_gaussians* g, const vcgs_views* views, const float bg[3],
                              const vcgs_images* outs, int flags, void* stream)
{
    return render_batch_impl(ctx, g, views, bg, nullptr, nullptr, 0.0f, outs, nullptr, nullptr, nullptr, flags,
                             nullptr, true, stream);
}

int vcgs_render_batch_backward(vcgs_ctx* ctx, const vcgs_gaussians* g, const vcgs_views* views,
                               const float* const* dl_dcolor, const float* const* dl_ddepth,
                               const float* const* dl_dalpha, vcgs_gaussian_buffers* grads, float* dl_dpose,
                               int flags, void* stream)
{
    if (!ctx || !views) return fail(VCGS_E_INVALID, "ctx or views is NULL");
    BatchPlan* p = ctx->fwd_plan;
    if (!p) return fail(VCGS_E_INVALID, "no batched forward (vcgs_render_batch_forward) to differentiate");
    const int V = views->n_views;
    int rc;
    if ((rc = check_gaussians(g, std::max(V, 1))) != VCGS_OK) return rc;
    if (V != p->V || g->n != p->n || flags != p->flags || !views->cams || !views->poses)
        return fail(VCGS_E_INVALID, "views, Gaussian count or flags differ from the last batched forward");
    const void* gp[5] = {g->mean, g->scale, g->quat, g->opacity, g->color};
    for (int i = 0; i < 5; ++i)
        if (p->ptrs[i] != gp[i]) return fail(VCGS_E_INVALID, "Gaussians differ from the last batched forward");
    for (int v = 0; v < V; ++v) {
        if (std::memcmp(&p->cams[v], &views->cams[v], sizeof(vcgs_camera)) != 0)
            return fail(VCGS_E_INVALID, "cameras differ from the last batched forward");
        const PoseK pk = make_posek(views->poses[v]);
        if (std::memcmp(&pk, &p->f.pt.pose[v], sizeof(PoseK)) != 0)
            return fail(VCGS_E_INVALID, "poses differ from the last batched forward");
    }
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(hipSetDevice(ctx->device));
    if (!p->g2) {
        p->pb = std::max(1, preprocess_bwd_blocks(p->f.n));
        p->g2 = p->get_e<float>((int64_t)kG2 * p->f.E);
        p->partial = p->get_e<float>(6 * (int64_t)p->pb * V);
        if (!p->ok()) {
            // the failed blocks stay listed (null) until the plan is released; later calls refuse
            return fail(VCGS_E_NOMEM, "allocation failed (batch backward)");
        }
        // later forwards zero the gradient slots in their projection (a
        // captured forward without them is captured again)
        p->f.g2 = p->g2;
        if (p->exec) {
            HIP_TRY(hipStreamSynchronize(s));
            p->drop_graph();
        }
    }
    if (!p->ok()) return fail(VCGS_E_NOMEM, "allocation failed (batch backward)");
    const vcgs_gaussian_buffers gb =
        grads ? *grads : vcgs_gaussian_buffers{nullptr, nullptr, nullptr, nullptr, nullptr};
    Frame fb = p->f;  // the forward's tables with this call's upstream gradients
    std::vector<const void*> key = {gb.mean, gb.scale, gb.quat, gb.opacity, gb.color, dl_dpose};
    for (int v = 0; v < V; ++v) {
        fb.vt.dl_dc[v] = dl_dcolor ? dl_dcolor[v] : nullptr;
        fb.vt.dl_dd[v] = dl_ddepth ? dl_ddepth[v] : nullptr;
        fb.vt.dl_da[v] = dl_dalpha ? dl_dalpha[v] : nullptr;
        key.push_back(fb.vt.dl_dc[v]);
        key.push_back(fb.vt.dl_dd[v]);
        key.push_back(fb.vt.dl_da[v]);
    }
    // the gradient slots start at zero: zeroed by the forward's projection, or
    // here (first backward after a forward without them, or a second backward)
    if (!p->g2_zeroed) launch_fill_f32(p->g2, 0.0f, (int64_t)kG2 * p->f.E, s);
    p->g2_zeroed = false;
    if (flags & VCGS_BATCH_GRAPH) {
        if (!ctx->graph_stream) HIP_TRY(hipStreamCreateWithFlags(&ctx->graph_stream, hipStreamNonBlocking));
        hipStream_t gs = ctx->graph_stream;
        if (!p->exec_bwd || p->bwd_ptrs != key) {
            if (p->exec_bwd) (void)hipGraphExecDestroy(p->exec_bwd);
            if (p->graph_bwd) (void)hipGraphDestroy(p->graph_bwd);
            p->exec_bwd = nullptr;
            p->graph_bwd = nullptr;
            HIP_TRY(hipStreamSynchronize(s));
            ctx->prof.capturing = true;
            hipError_t e = hipStreamBeginCapture(gs, hipStreamCaptureModeThreadLocal);
            if (e == hipSuccess) {
                backward_core(ctx, fb, *g, gb, dl_dpose, p->g2, p->partial, p->pb, gs, false);
                e = hipStreamEndCapture(gs, &p->graph_bwd);
            }
            ctx->prof.capturing = false;
            if (e == hipSuccess) e = hipGraphInstantiate(&p->exec_bwd, p->graph_bwd, nullptr, nullptr, 0);
            if (e != hipSuccess) {
                if (p->graph_bwd) (void)hipGraphDestroy(p->graph_bwd);
                p->graph_bwd = nullptr;
                p->exec_bwd = nullptr;
                return fail(VCGS_E_HIP, std::string("graph capture failed: ") + hipGetErrorString(e));
            }
            p->bwd_ptrs = key;
        }
        HIP_TRY(hipGraphLaunch(p->exec_bwd, s));
    } else {
        backward_core(ctx, fb, *g, gb, dl_dpose, p->g2, p->partial, p->pb, s, false);
    }
    ctx->last_stream = s;
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(VCGS_E_HIP, std::string("kernel launch failed: ") + hipGetErrorString(e));
    return VCGS_OK;
}

int vcgs_batch_check(vcgs_ctx* ctx, int64_t* pairs)
{
    if (!ctx) return fail(VCGS_E_INVALID, "ctx is NULL");
    if (pairs) *pairs = 0;
    BatchPlan* p = ctx->last_plan;
    if (!p) return VCGS_OK;
    HIP_TRY(hipSetDevice(ctx->device));
    HIP_TRY(hipStreamSynchronize(ctx->last_stream));
    // pair total of the last pass and the sticky overflow word are adjacent
    HIP_TRY(hipMemcpy(p->host_flags, p->w.total, 2 * sizeof(uint32_t), hipMemcpyDeviceToHost));
    const int64_t total = p->host_flags[0];
    const int64_t over = p->host_flags[1];
    if (pairs) *pairs = total;
    if (over != 0) {
        p->need = over;
        ctx->last_required_pairs = over;
        launch_fill_u32(p->w.overflow, 0u, 1, ctx->last_stream);
        HIP_TRY(hipStreamSynchronize(ctx->last_stream));
        return fail(VCGS_E_CAPACITY, "pair buffer of a batched pass was too small (" + std::to_string(over) +
                                         " pairs needed); the next call resizes it, rerun the pass");
    }
    return VCGS_OK;
}

int64_t vcgs_last_required_pairs(const vcgs_ctx* ctx)
{
    return ctx ? ctx->last_required_pairs : 0;
}

void vcgs_camera_centres(int n_views, const vcgs_pose* poses, float* centres)
{
    // paper eq. (9): the camera centre of a world-to-camera pose {R|t} is -R^T t
    for (int v = 0; poses && centres && v < n_views; ++v) {
        const float* R = poses[v].R;
        const float* t = poses[v].t;
        for (int i = 0; i < 3; ++i)
            centres[3 * v + i] = (float)(-((double)R[i] * t[0] + (double)R[3 + i] * t[1] + (double)R[6 + i] * t[2]));
    }
}

}  // extern "C"
