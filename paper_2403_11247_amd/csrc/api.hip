// C ABI of the vcgs library: contexts, errors, anchor decode, loss, kernel
// options and stage timing.  The render entry points are in frame.hip.
#include <cmath>
#include <cstdio>

#include "ctx.h"

using namespace vcgs;

namespace vcgs {
thread_local std::string g_err;
}  // namespace vcgs

extern "C" {

const char* vcgs_last_error(void) { return g_err.c_str(); }
const char* vcgs_version(void) { return "vcgs 0.2 gfx950"; }

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
    int rc = noalloc_init(device);
    if (rc != VCGS_OK) return rc;
    vcgs_ctx* c = new vcgs_ctx();
    c->device = device;
    c->pool.dev = &c->dalloc;
    if (hipHostMalloc((void**)&c->host_u32, 64, hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void**)&c->host_tab, sizeof(ProjTab), hipHostMallocDefault) != hipSuccess ||
        hipEventCreateWithFlags(&c->graph_done, hipEventDisableTiming) != hipSuccess) {
        if (c->host_u32) (void)hipHostFree(c->host_u32);
        if (c->host_tab) (void)hipHostFree(c->host_tab);
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
    destroy_plans(ctx);
    ctx->prof.destroy();
    if (ctx->prof.d_counters) (void)hipFree(ctx->prof.d_counters);
    ctx->pool.destroy();
    if (ctx->host_u32) (void)hipHostFree(ctx->host_u32);
    if (ctx->host_tab) (void)hipHostFree(ctx->host_tab);
    if (ctx->graph_done) (void)hipEventDestroy(ctx->graph_done);
    delete ctx;
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

}  // extern "C"

namespace vcgs {
int make_decode_args(const vcgs_anchors* a, const vcgs_mlp* mlp, const vcgs_codebook* cb, const float* mask_logit,
                     float mask_eps, DecodeArgs* d, const float* cam, int views)
{
    if (views < 1 || views > kDecodeMaxViews || (!cam && views != 1))
        return fail(VCGS_E_INVALID, "views must be in [1, 16] (and 1 without camera centres)");
    d->in_dim = cam ? 36 : 32;
    d->views = views;
    for (int v = 0; v < kDecodeMaxViews; ++v)
        for (int i = 0; i < 3; ++i) d->cam[v][i] = (cam && v < views) ? cam[3 * v + i] : 0.0f;
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
}  // namespace vcgs

extern "C" {

static int decode_fwd(vcgs_ctx* ctx, const vcgs_anchors* a, const vcgs_mlp* mlp, const vcgs_codebook* cb,
                      const float* mask_logit, float mask_eps, const float* cam, int views,
                      vcgs_gaussian_buffers* out, void* stream)
{
    if (!ctx || !out) return fail(VCGS_E_INVALID, "ctx or out is NULL");
    DecodeArgs d;
    int rc = make_decode_args(a, mlp, cb, mask_logit, mask_eps, &d, cam, views);
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

static int decode_bwd(vcgs_ctx* ctx, const vcgs_anchors* a, const vcgs_mlp* mlp, const vcgs_codebook* cb,
                      const float* mask_logit, float mask_eps, const float* cam, int views,
                      const vcgs_gaussian_buffers* dG, vcgs_anchor_grads* out, void* stream)
{
    if (!ctx || !out || !dG) return fail(VCGS_E_INVALID, "ctx, dG or out is NULL");
    DecodeArgs d;
    int rc = make_decode_args(a, mlp, cb, mask_logit, mask_eps, &d, cam, views);
    if (rc != VCGS_OK) return rc;
    HIP_TRY(hipSetDevice(ctx->device));
    hipStream_t s = (hipStream_t)stream;
    vcgs_anchor_grads o = *out;
    if (!cb) o.books = nullptr;
    if (!mask_logit) o.mask_logit = nullptr;
    if (!cam) o.cam = nullptr;
    if (d.na == 0) {  // no anchors: the weight, codebook and centre gradients are zero
        const int O = d.k * 11;
        if (o.W1) launch_fill_f32(o.W1, 0.0f, 32 * d.in_dim, s);
        if (o.b1) launch_fill_f32(o.b1, 0.0f, 32, s);
        if (o.W2) launch_fill_f32(o.W2, 0.0f, (int64_t)O * 32, s);
        if (o.b2) launch_fill_f32(o.b2, 0.0f, O, s);
        if (o.books) launch_fill_f32(o.books, 0.0f, (int64_t)d.stages * d.cb_size * 7, s);
        if (o.cam) launch_fill_f32(o.cam, 0.0f, 3 * d.views, s);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return fail(VCGS_E_HIP, std::string("kernel launch failed: ") + hipGetErrorString(e));
        return VCGS_OK;
    }
    Scratch sc(&ctx->pool);
    const int nb = decode_bwd_blocks(d.na, d.k);
    float* partial = sc.get<float>((int64_t)nb * decode_bwd_partial_floats(d.k, d.in_dim, d.views));
    float *dvbuf = nullptr, *book_partial = nullptr;
    if (o.books && (size_t)d.cb_size * 7 * sizeof(float) <= kBookLdsMax) {
        const int64_t ng = d.na * d.k;
        dvbuf = sc.get<float>(ng * 8);
        book_partial = sc.get<float>((int64_t)books_grad_blocks(ng) * d.stages * d.cb_size * 7);
    }
    if (sc.oom) return fail(VCGS_E_NOMEM, "device allocation failed (decode backward)");
    ctx->prof.begin(VCGS_STAGE_DECODE_BWD, s);
    launch_decode_bwd(d, *dG, o, partial, nb, dvbuf, book_partial, s);
    ctx->prof.end(VCGS_STAGE_DECODE_BWD, s);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(VCGS_E_HIP, std::string("kernel launch failed: ") + hipGetErrorString(e));
    return VCGS_OK;
}

int vcgs_decode_anchors(vcgs_ctx* ctx, const vcgs_anchors* a, const vcgs_mlp* mlp, const vcgs_codebook* cb,
                        const float* mask_logit, float mask_eps, vcgs_gaussian_buffers* out, void* stream)
{
    return decode_fwd(ctx, a, mlp, cb, mask_logit, mask_eps, nullptr, 1, out, stream);
}

int vcgs_decode_anchors_backward(vcgs_ctx* ctx, const vcgs_anchors* a, const vcgs_mlp* mlp, const vcgs_codebook* cb,
                                 const float* mask_logit, float mask_eps, const vcgs_gaussian_buffers* dG,
                                 vcgs_anchor_grads* out, void* stream)
{
    return decode_bwd(ctx, a, mlp, cb, mask_logit, mask_eps, nullptr, 1, dG, out, stream);
}

int vcgs_decode_anchors_view(vcgs_ctx* ctx, const vcgs_anchors* a, const vcgs_mlp* mlp, const vcgs_codebook* cb,
                             const float* mask_logit, float mask_eps, const float cam_centre[3],
                             vcgs_gaussian_buffers* out, void* stream)
{
    if (!cam_centre) return fail(VCGS_E_INVALID, "cam_centre is NULL");
    return decode_fwd(ctx, a, mlp, cb, mask_logit, mask_eps, cam_centre, 1, out, stream);
}

int vcgs_decode_anchors_views(vcgs_ctx* ctx, const vcgs_anchors* a, const vcgs_mlp* mlp, const vcgs_codebook* cb,
                              const float* mask_logit, float mask_eps, int n_views, const float* cam_centres,
                              vcgs_gaussian_buffers* out, void* stream)
{
    if (!cam_centres) return fail(VCGS_E_INVALID, "cam_centres is NULL");
    return decode_fwd(ctx, a, mlp, cb, mask_logit, mask_eps, cam_centres, n_views, out, stream);
}

int vcgs_decode_anchors_view_backward(vcgs_ctx* ctx, const vcgs_anchors* a, const vcgs_mlp* mlp,
                                      const vcgs_codebook* cb, const float* mask_logit, float mask_eps,
                                      const float cam_centre[3], const vcgs_gaussian_buffers* dG,
                                      vcgs_anchor_grads* out, void* stream)
{
    if (!cam_centre) return fail(VCGS_E_INVALID, "cam_centre is NULL");
    return decode_bwd(ctx, a, mlp, cb, mask_logit, mask_eps, cam_centre, 1, dG, out, stream);
}

int vcgs_decode_anchors_views_backward(vcgs_ctx* ctx, const vcgs_anchors* a, const vcgs_mlp* mlp,
                                       const vcgs_codebook* cb, const float* mask_logit, float mask_eps,
                                       int n_views, const float* cam_centres, const vcgs_gaussian_buffers* dG,
                                       vcgs_anchor_grads* out, void* stream)
{
    if (!cam_centres) return fail(VCGS_E_INVALID, "cam_centres is NULL");
    return decode_bwd(ctx, a, mlp, cb, mask_logit, mask_eps, cam_centres, n_views, dG, out, stream);
}

int vcgs_centre_pose_grad(vcgs_ctx* ctx, int n_views, const vcgs_pose* poses, const float* dcam, float* dpose,
                          void* stream)
{
    if (!ctx || !poses || (n_views > 0 && (!dcam || !dpose)))
        return fail(VCGS_E_INVALID, "ctx, poses, dcam or dpose is NULL");
    if (n_views < 0 || n_views > kDecodeMaxViews) return fail(VCGS_E_INVALID, "n_views must be in [0, 16]");
    CentreTab t;
    t.views = n_views;
    for (int v = 0; v < n_views; ++v)
        for (int k = 0; k < 9; ++k) t.R[v][k] = poses[v].R[k];
    HIP_TRY(hipSetDevice(ctx->device));
    launch_centre_pose_grad(t, dcam, dpose, (hipStream_t)stream);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(VCGS_E_HIP, std::string("kernel launch failed: ") + hipGetErrorString(e));
    return VCGS_OK;
}

int vcgs_mask_loss(vcgs_ctx* ctx, int64_t n, const float* mask_logit, const uint32_t* in_frustum_count,
                   float weight, float* dl_dm, float* loss, void* stream)
{
    if (!ctx) return fail(VCGS_E_INVALID, "ctx is NULL");
    if (n < 0) return fail(VCGS_E_INVALID, "negative Gaussian count");
    if (n > 0 && !mask_logit) return fail(VCGS_E_INVALID, "mask_logit is NULL");
    HIP_TRY(hipSetDevice(ctx->device));
    hipStream_t s = (hipStream_t)stream;
    Scratch sc(&ctx->pool);
    float* partial = sc.get<float>(2 * (int64_t)mask_loss_blocks(n) + 1);
    if (sc.oom) return fail(VCGS_E_NOMEM, "device allocation failed (mask loss)");
    launch_mask_loss(n, mask_logit, in_frustum_count, weight, dl_dm, loss, partial, s);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(VCGS_E_HIP, std::string("kernel launch failed: ") + hipGetErrorString(e));
    return VCGS_OK;
}

int vcgs_mask_prune(vcgs_ctx* ctx, int64_t n, const float* mask_logit, float mask_eps, const uint32_t* hits,
                    uint32_t min_hits, uint8_t* keep, uint32_t* kept_index, int64_t* n_kept, void* stream)
{
    if (!ctx || !n_kept) return fail(VCGS_E_INVALID, "ctx or n_kept is NULL");
    if (n < 0 || n > kMaxSortItems) return fail(VCGS_E_INVALID, "n must be in [0, 2^30)");
    if (n > 0 && !mask_logit) return fail(VCGS_E_INVALID, "mask_logit is NULL");
    if (!(mask_eps > 0.0f && mask_eps < 1.0f)) return fail(VCGS_E_INVALID, "mask_eps must be in (0, 1)");
    HIP_TRY(hipSetDevice(ctx->device));
    hipStream_t s = (hipStream_t)stream;
    Scratch sc(&ctx->pool);
    uint32_t* flags = sc.get<uint32_t>(n);
    uint32_t* offs = sc.get<uint32_t>(n);
    uint32_t* cnt = sc.get<uint32_t>(4);
    uint32_t* tmp = sc.get<uint32_t>(scan_temp_words(n) + 8);
    if (sc.oom) return fail(VCGS_E_NOMEM, "device allocation failed (prune)");
    const float thr = (float)std::log((double)mask_eps / (1.0 - (double)mask_eps));
    launch_mask_prune(n, mask_logit, thr, hits, min_hits, keep, flags, offs, kept_index, cnt, tmp, s);
    HIP_TRY(hipMemcpyAsync(ctx->host_u32, cnt, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    *n_kept = ctx->host_u32[0];
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
    case VCGS_OPT_BWD_MERGE:
        if (value != 0 && value != 1) return fail(VCGS_E_INVALID, "bwd_merge must be 0 or 1");
        o.bwd_merge = value;
        return VCGS_OK;
    case VCGS_OPT_SCHED:
        if (value != 0 && value != 1) return fail(VCGS_E_INVALID, "sched must be 0 or 1");
        o.sched = value;
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
    case VCGS_OPT_SCHED: *value = o.sched; return VCGS_OK;
    case VCGS_OPT_BWD_MERGE: *value = o.bwd_merge; return VCGS_OK;
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

int vcgs_profile_stages(vcgs_ctx* ctx, uint32_t mask)
{
    if (!ctx) return fail(VCGS_E_INVALID, "ctx is NULL");
    ctx->prof.mask = mask;
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

int vcgs_rvq_assign(vcgs_ctx* ctx, const vcgs_rvq_books* q, int64_t n, const float* x, void* idx, int32_t idx_bytes,
                    float* recon, float* loss, float* dbooks, void* stream)
{
    if (!ctx || !q) return fail(VCGS_E_INVALID, "ctx or q is NULL");
    const int D = q->dim, L = q->stages, P = q->codes;
    if (D < 1 || D > 32 || L < 1 || L > 8 || P < 1 || P > 256)
        return fail(VCGS_E_INVALID, "R-VQ needs 1 <= dim <= 32, 1 <= stages <= 8, 1 <= codes <= 256");
    if (dbooks && (int64_t)L * P * ((D + 1) | 1) > 16384)
        return fail(VCGS_E_INVALID, "stages * codes * ((dim + 1) | 1) exceeds 16384 with a code gradient");
    if (!q->books) return fail(VCGS_E_INVALID, "books is NULL");
    if (n < 0 || n > ((int64_t)1 << 40)) return fail(VCGS_E_INVALID, "n out of range");
    if (n > 0 && !x) return fail(VCGS_E_INVALID, "x is NULL");
    if (idx && idx_bytes != 1 && idx_bytes != 4) return fail(VCGS_E_INVALID, "idx_bytes must be 1 or 4");
    HIP_TRY(hipSetDevice(ctx->device));
    hipStream_t s = (hipStream_t)stream;
    Scratch sc(&ctx->pool);
    float* tab = sc.get<float>((int64_t)L * P * (rvq_padded_dim(D) + 4));
    const bool grad = dbooks != nullptr;
    float* partial = (loss || grad) ? sc.get<float>(rvq_partial_floats(n, L, P, D, grad)) : nullptr;
    double* red = (loss || grad) ? sc.get<double>(rvq_red_doubles(n, L, P, D, grad)) : nullptr;
    if (sc.oom) return fail(VCGS_E_NOMEM, "device allocation failed (R-VQ)");
    if (!launch_rvq(n, D, L, P, q->books, x, idx, idx_bytes, recon, loss, dbooks, tab, partial, red, s))
        return fail(VCGS_E_UNSUPPORTED, "the device refused the LDS size this R-VQ launch needs");
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(VCGS_E_HIP, std::string("kernel launch failed: ") + hipGetErrorString(e));
    return VCGS_OK;
}

int vcgs_track_loss(vcgs_ctx* ctx, const vcgs_images* img, const float* target_color, const float* target_depth,
                    int32_t width, int32_t height, float lam_d, int32_t norm, float sil_thresh, float* dl_dcolor,
                    float* dl_ddepth, float* loss, void* stream)
{
    if (!ctx || !img) return fail(VCGS_E_INVALID, "ctx or img is NULL");
    if (width <= 0 || height <= 0 || (int64_t)width * height > ((int64_t)1 << 31))
        return fail(VCGS_E_INVALID, "image size out of range");
    if (!img->color || !img->depth || !img->alpha || !target_color || !target_depth)
        return fail(VCGS_E_INVALID, "an image is NULL (colour, depth, silhouette and both targets are needed)");
    if (norm != 1 && norm != 2) return fail(VCGS_E_INVALID, "norm must be 1 or 2");
    if ((dl_dcolor == nullptr) != (dl_ddepth == nullptr))
        return fail(VCGS_E_INVALID, "dl_dcolor and dl_ddepth go together");
    HIP_TRY(hipSetDevice(ctx->device));
    hipStream_t s = (hipStream_t)stream;
    Scratch sc(&ctx->pool);
    float* partial = sc.get<float>(track_partial_floats(width, height));
    if (sc.oom) return fail(VCGS_E_NOMEM, "device allocation failed (track loss)");
    launch_track_loss(width, height, img->color, img->depth, img->alpha, target_color, target_depth, lam_d, norm,
                      sil_thresh, dl_dcolor, dl_ddepth, loss, partial, s);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(VCGS_E_HIP, std::string("kernel launch failed: ") + hipGetErrorString(e));
    return VCGS_OK;
}

int vcgs_icp_loss(vcgs_ctx* ctx, int64_t n, const float* mean, const vcgs_camera* cam, const vcgs_pose* pose,
                  const float* depth, float tau, int32_t stride, float weight, float* dmean, float* dpose,
                  float* loss, uint32_t* matched, void* stream)
{
    if (!ctx || !cam || !pose) return fail(VCGS_E_INVALID, "ctx, cam or pose is NULL");
    if (n < 0 || n > kMaxSortItems) return fail(VCGS_E_INVALID, "n must be in [0, 2^30)");
    if (n > 0 && (!mean || !depth)) return fail(VCGS_E_INVALID, "mean or depth is NULL");
    if (cam->width <= 0 || cam->height <= 0 || !(cam->fx > 0.0f) || !(cam->fy > 0.0f))
        return fail(VCGS_E_INVALID, "camera needs a positive size and focal lengths");
    if (!(tau > 0.0f) || stride < 1) return fail(VCGS_E_INVALID, "tau must be > 0 and stride >= 1");
    HIP_TRY(hipSetDevice(ctx->device));
    hipStream_t s = (hipStream_t)stream;
    Scratch sc(&ctx->pool);
    float* partial = sc.get<float>(8 * (int64_t)icp_blocks(n) + 8);
    float* tmin = sc.get<float>(icp_tile_floats(cam->width, cam->height));
    if (sc.oom) return fail(VCGS_E_NOMEM, "device allocation failed (ICP)");
    launch_icp(n, mean, depth, cam->width, cam->height, cam->fx, cam->fy, cam->cx, cam->cy, pose->R, pose->t, tau,
               stride, weight, dmean, loss, dpose, matched, partial, tmin, s);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(VCGS_E_HIP, std::string("kernel launch failed: ") + hipGetErrorString(e));
    return VCGS_OK;
}

int vcgs_ssim_loss(vcgs_ctx* ctx, const float* color, const float* target_color, int32_t width, int32_t height,
                   float weight, float* dl_dcolor, float* loss, void* stream)
{
    if (!ctx) return fail(VCGS_E_INVALID, "ctx is NULL");
    if (width <= 0 || height <= 0 || (int64_t)width * height > ((int64_t)1 << 29))
        return fail(VCGS_E_INVALID, "image size out of range");
    if (!color || !target_color) return fail(VCGS_E_INVALID, "an image is NULL");
    HIP_TRY(hipSetDevice(ctx->device));
    hipStream_t s = (hipStream_t)stream;
    Scratch sc(&ctx->pool);
    float* dm = sc.get<float>(9 * (int64_t)width * height);
    float* partial = sc.get<float>(ssim_partial_floats(width, height));
    if (sc.oom) return fail(VCGS_E_NOMEM, "device allocation failed (SSIM)");
    launch_ssim_loss(width, height, color, target_color, weight, dl_dcolor, loss, dm, partial, s);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(VCGS_E_HIP, std::string("kernel launch failed: ") + hipGetErrorString(e));
    return VCGS_OK;
}

int vcgs_set_allocator(vcgs_ctx* ctx, vcgs_alloc_fn alloc, vcgs_free_fn free_fn, void* user)
{
    if (!ctx) return fail(VCGS_E_INVALID, "ctx is NULL");
    if ((alloc == nullptr) != (free_fn == nullptr)) return fail(VCGS_E_INVALID, "alloc and free go together");
    if (ctx->servers > 0) return fail(VCGS_E_INVALID, "a server of this context is alive");
    HIP_TRY(hipSetDevice(ctx->device));
    destroy_plans(ctx);
    ctx->pool.release_cache();
    if (!ctx->pool.sizes.empty()) return fail(VCGS_E_INVALID, "workspaces are in use (a render state is alive)");
    ctx->dalloc.alloc_fn = alloc;
    ctx->dalloc.free_fn = free_fn;
    ctx->dalloc.user = user;
    return VCGS_OK;
}

}  // extern "C"
