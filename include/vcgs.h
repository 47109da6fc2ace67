/*
 * vcgs -- differentiable tile-based Gaussian rasterizer for voxel-anchored
 * compact 3D Gaussian SLAM (arXiv 2403.11247), native on AMD Instinct MI355X
 * (gfx950).
 *
 * C ABI.  Every pointer argument that names image, Gaussian, anchor, weight or
 * gradient data is a DEVICE pointer owned by the caller; the library never
 * frees caller memory.  Structs passed by pointer (cameras, poses, the
 * descriptors below) live in HOST memory and are read during the call only.
 * Every call enqueues work on the caller's `stream` (hipStream_t passed as
 * void*) and returns before the GPU finishes unless stated otherwise.
 * Return value: VCGS_OK (0) or a negative VCGS_E_* code; the message of the
 * last failing call on the calling thread is returned by vcgs_last_error().
 * A context serves one device; calls on one context must not overlap in time
 * from different host threads.
 *
 * Array layouts (float32 unless noted; n = number of Gaussians):
 *   mean [3][n], scale [3][n] (linear, not log), quat [4][n] (w, x, y, z; need
 *   not be unit: the renderer normalises it, a zero quaternion means identity),
 *   opacity [n], color [3][n];
 *   images: color [3][H][W], depth [H][W], alpha [H][W] (row-major, x fastest).
 */
#ifndef VCGS_H
#define VCGS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    VCGS_OK = 0,
    VCGS_E_INVALID = -1,      /* bad argument: null pointer, negative size, unsupported tile size */
    VCGS_E_NOMEM = -2,        /* device allocation failed */
    VCGS_E_CAPACITY = -3,     /* a fixed-capacity buffer was too small (batched/captured mode) */
    VCGS_E_HIP = -4,          /* a HIP runtime call failed (message holds the HIP error string) */
    VCGS_E_UNSUPPORTED = -5   /* device is not gfx950 or the request exceeds a documented limit */
};

typedef struct vcgs_ctx vcgs_ctx;
typedef struct vcgs_state vcgs_state;

/* Pinhole camera with known intrinsics K (paper Sec. 3: RGB-D frames with known
 * K).  Pixel (x, y) is sampled at (x + 0.5, y + 0.5).  z_near culls Gaussians
 * whose mean is not in front of the camera.  tile must be 16. */
typedef struct {
    int32_t width, height;
    float fx, fy, cx, cy;
    float z_near;
    int32_t tile;
} vcgs_camera;

/* Camera pose {R|t} (paper Sec. 3), world to camera: p_cam = R p_world + t.
 * R row-major.  The camera looks along +z, x right, y down. */
typedef struct {
    float R[9];
    float t[3];
} vcgs_pose;

/* Gaussian attributes (paper Sec. 3.2: position, opacity, quaternion, scaling, colour). */
typedef struct {
    int64_t n;
    const float* mean;
    const float* scale;
    const float* quat;
    const float* opacity;
    const float* color;
} vcgs_gaussians;

/* Writable Gaussian-shaped buffers: decode output, or gradients. */
typedef struct {
    float* mean;
    float* scale;
    float* quat;
    float* opacity;
    float* color;
} vcgs_gaussian_buffers;

typedef struct {
    float* color;  /* [3][H][W]  eq. (16) plus T_final * background */
    float* depth;  /* [H][W]     eq. (17), not normalised */
    float* alpha;  /* [H][W]     eq. (18), the silhouette S(p) */
} vcgs_images;

/* ---- context ---------------------------------------------------------- */

/* Create a context on HIP device `device`.  Fails with VCGS_E_UNSUPPORTED if
 * the device is not gfx950. */
int vcgs_create(int device, vcgs_ctx** out);
void vcgs_destroy(vcgs_ctx* ctx);
/* Message of the last failing call on this host thread ("" if none). */
const char* vcgs_last_error(void);
/* Library version string. */
const char* vcgs_version(void);

/* Device memory of the context's workspaces, render states, batch plans and
 * servers: from hipMalloc / hipFree (the default, alloc = free = NULL), or
 * from the caller's functions, e.g. a framework's caching allocator.  alloc
 * returns a device pointer of at least `bytes` (NULL = out of memory); free
 * takes it back.  The library returns memory only after the work that used it
 * has finished (it synchronises first), so the caller may reuse it at once.
 * Call it before the context holds memory: it drops the context's batch plans
 * and cached blocks, and fails with VCGS_E_INVALID while a render state or a
 * server of the context is alive. */
typedef void* (*vcgs_alloc_fn)(size_t bytes, void* user);
typedef void (*vcgs_free_fn)(void* ptr, void* user);
int vcgs_set_allocator(vcgs_ctx* ctx, vcgs_alloc_fn alloc, vcgs_free_fn free_fn, void* user);

/* ---- plain render ----------------------------------------------------- */

/* Forward render of one view (paper eqs. (1)-(3) and (16)-(18)).
 *   Projects every Gaussian (EWA, eq. (3) with W = R), bins it to the 16x16
 *   tiles its footprint can reach, sorts the (tile, depth) pairs (stable: equal
 *   keys keep Gaussian index order), and composites each pixel front to back:
 *     alpha_i = min(0.99, o_i exp(-1/2 d^T Q_i d)), skipped when < 1/255;
 *     stops before the Gaussian that would take the transmittance below 1e-4;
 *     C = sum c_i alpha_i T_i + T_final bg, D = sum z_i alpha_i T_i, A = sum alpha_i T_i.
 *   bg: 3 floats in HOST memory.  out: device images of the camera's size.
 *   state: if non-NULL, receives a new saved-for-backward object (free with
 *   vcgs_state_free).  The call synchronises `stream` once, after binning, to
 *   size the pair buffers.
 */
int vcgs_render_forward(vcgs_ctx* ctx, const vcgs_gaussians* g, const vcgs_camera* cam,
                        const vcgs_pose* pose, const float bg[3], vcgs_images* out,
                        vcgs_state** state, void* stream);

/* Backward of vcgs_render_forward (paper Sec. 4: the renderer's backward
 * propagation extended to depth, pose and cumulative opacity).
 *   g, cam, pose, bg must be those of the forward call, unchanged.
 *   dl_dcolor [3][H][W], dl_ddepth [H][W], dl_dalpha [H][W]: device upstream
 *   gradients (any may be NULL = zero).
 *   grads: device buffers of the Gaussian shapes, OVERWRITTEN with dL/d(mean,
 *   scale, quat, opacity, color) (culled Gaussians get 0); any field may be NULL.
 *   dl_dpose: device float[6], OVERWRITTEN with dL/dxi for the left
 *   perturbation {R|t} <- exp(xi^) {R|t}, xi = (rho, phi) at 0; may be NULL.
 *   The compositing is replayed back to front from the saved final
 *   transmittance; no per-pixel lists are stored.
 */
int vcgs_render_backward(vcgs_ctx* ctx, const vcgs_state* state, const vcgs_gaussians* g,
                         const vcgs_camera* cam, const vcgs_pose* pose,
                         const float* dl_dcolor, const float* dl_ddepth, const float* dl_dalpha,
                         vcgs_gaussian_buffers* grads, float* dl_dpose, void* stream);

void vcgs_state_free(vcgs_ctx* ctx, vcgs_state* state);

/* Allocation-free forward render, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  Same arguments and images as vcgs_render_forward with
 * state = NULL, from the same kernels, but every buffer of the pass comes
 * from one fixed device array of VCGS_NOALLOC_SCRATCH_BYTES (128 MiB) per
 * GPU, held from the first vcgs_create on that GPU until the process ends;
 * the call makes no hipMalloc, hipFree or other allocating call.
 *   Sizes: the pass needs about 104 bytes per Gaussian, 8 per pixel and 16 per
 *   (tile, Gaussian) pair (one 1200x680 view of 400k Gaussians with 2.3M pairs
 *   takes about 85 MB).  A pass that does not fit returns VCGS_E_CAPACITY
 *   before any launch (Gaussians and pixels) or after the pair count is known
 *   (pairs; vcgs_last_required_pairs then holds the count); the output images
 *   are left unwritten.
 *   Like vcgs_render_forward it synchronises `stream` once, after binning.
 *   Every call on one GPU, from any context or thread, uses that GPU's one
 *   array and leaves its contents behind: calls that overlap in time on one
 *   GPU (other streams, other threads) race and must be serialised by the
 *   caller.  The kernels clear what they need before use. */
#define VCGS_NOALLOC_SCRATCH_BYTES ((size_t)128 << 20)
int vcgs_render_forward_noalloc(vcgs_ctx* ctx, const vcgs_gaussians* g, const vcgs_camera* cam,
                                const vcgs_pose* pose, const float bg[3], vcgs_images* out, void* stream);

/* Read-only view of a saved state, for inspection and tests.  Device pointers
 * stay valid until vcgs_state_free.
 *   depth_bits[n]  uint32 bits of the float camera depth (0xFFFFFFFF = culled)
 *   rect[n]        uint16 x4 (tx0, ty0, tx1, ty1) inclusive tile rectangle
 *   count[n]       uint32 number of tiles (0 = culled)
 *   gids[P]        Gaussian index of every (tile, depth)-sorted pair
 *   ranges[T][2]   [start, end) of each tile's pairs in gids
 *   t_final[H][W], n_contrib[H][W] (uint32: list entries up to the last contributor)
 *   splats[n][16]  float: u, v, u_lo, v_lo, s1 ex, s1 ey, s2 ex, s2 ey, opacity, r, g, b, depth,
 *                  s1, s2, 0 (visible Gaussians only): screen position u + u_lo, v + v_lo; unit
 *                  major axis (ex, ey); s = sqrt(1 / (2 ln2 lambda)) for the eigenvalues lambda1 >=
 *                  lambda2 of Sigma' + 0.3 I (the footprint is 2^-(q1^2 + q2^2) with
 *                  q1 = s1 d . (ex, ey), q2 = s2 d . (-ey, ex))
 */
typedef struct {
    int64_t n, n_pairs;
    int32_t tiles_x, tiles_y;
    const uint32_t* depth_bits;
    const uint16_t* rect;
    const uint32_t* count;
    const uint32_t* gids;
    const uint32_t* ranges;
    const float* t_final;
    const uint32_t* n_contrib;
    const float* splats;
} vcgs_state_view;
int vcgs_state_query(const vcgs_state* state, vcgs_state_view* out);

/* L1 loss used by tracking and bundle adjustment (paper eq. (19) uses squared
 * errors; the L1 form with depth weight w_depth is the workload's):
 *   L = mean_p sum_c |C - C*| + w_depth mean_p |D - D*|.
 * Writes dl_dcolor, dl_ddepth (device, image shapes; subgradient 0 at equality)
 * and, if loss is non-NULL, the scalar loss (device float, overwritten). */
int vcgs_l1_loss(vcgs_ctx* ctx, const vcgs_images* img, const float* target_color,
                 const float* target_depth, int32_t width, int32_t height, float w_depth,
                 float* dl_dcolor, float* dl_ddepth, float* loss, void* stream);

/* ---- batched views ---------------------------------------------------- */

/* A set of views of one Gaussian map: cams, poses are HOST arrays of n_views. */
typedef struct {
    int32_t n_views;  /* 1..16 */
    const vcgs_camera* cams;
    const vcgs_pose* poses;
} vcgs_views;

/* VCGS_BATCH_GRAPH: capture the pass in a hipGraph and replay it.
 * VCGS_BATCH_PER_VIEW: every view has its own Gaussian set (e.g. the
 * view-dependent decode of paper eqs. (8)-(9), decoded once per keyframe):
 * g->n is the count per view and each attribute array holds the views' sets
 * one after another, each an ordinary SoA set (mean [V][3][n], quat
 * [V][4][n], opacity [V][n], ...); grads have the same layout and receive
 * each view's gradients separately instead of their sum. */
enum { VCGS_BATCH_GRAPH = 1, VCGS_BATCH_PER_VIEW = 2 };

/* Render n_views views of the same Gaussians in one pass (the keyframes of a
 * local bundle-adjustment window, paper Sec. 3.5, or the requests of one
 * serving step), and optionally run the loss and the backward for all of them.
 * This is the convenience form with the workload's L1 loss built in; the loss
 * stays outside the library with vcgs_render_batch_forward / _backward below.
 *   outs: HOST array of n_views device image sets (sizes of each camera).
 *   Forward only: target_color = target_depth = grads = dl_dpose = loss = NULL.
 *   Forward + backward: target_color / target_depth are HOST arrays of
 *   n_views device images; the L1 loss of vcgs_l1_loss (weight w_depth) is
 *   applied per view, loss (device float [n_views]) receives each view's loss
 *   if non-NULL, grads (device, Gaussian shapes) are OVERWRITTEN with the
 *   gradients summed over the views, dl_dpose (device float [n_views][6]) with
 *   each view's pose gradient (as in vcgs_render_backward).
 * Results equal those of per-view vcgs_render_forward / vcgs_l1_loss /
 * vcgs_render_backward calls up to the order of floating-point sums.
 * The first call with a given signature (sizes, intrinsics, flags and every
 * pointer argument) prepares a plan: it allocates the pass's buffers and
 * synchronises `stream` once to size the pair buffers with headroom.  Later
 * calls with the same signature (poses and Gaussian values may change) reuse
 * it without synchronising or reading anything back.  With VCGS_BATCH_GRAPH
 * the whole pass is captured once into a hipGraph (on a library-owned stream
 * ordered after `stream`) and replayed as one launch.  If the pairs of a pass
 * outgrow the buffers, the pass writes only what fits and the plan keeps, on
 * the device, the largest pair count any pass needed; vcgs_batch_check
 * reports it (VCGS_E_CAPACITY), the next call resizes, and the passes since
 * the previous check must be rerun. */
int vcgs_render_batch(vcgs_ctx* ctx, const vcgs_gaussians* g, const vcgs_views* views, const float bg[3],
                      const float* const* target_color, const float* const* target_depth, float w_depth,
                      const vcgs_images* outs, vcgs_gaussian_buffers* grads, float* dl_dpose, float* loss,
                      int flags, void* stream);

/* Batched pass with the loss outside the library (paper Sec. 3.5: the
 * bundle-adjustment loss is the tracking-like colour/depth term plus SSIM,
 * summed over the window's keyframes).  vcgs_render_batch_forward renders the
 * views as vcgs_render_batch does (same plans, capacity handling and graph
 * replay) and keeps the pass for one vcgs_render_batch_backward; the caller
 * computes the per-view upstream gradients from outs in between (e.g. with
 * vcgs_l1_loss, vcgs_track_loss, vcgs_ssim_loss). */
int vcgs_render_batch_forward(vcgs_ctx* ctx, const vcgs_gaussians* g, const vcgs_views* views, const float bg[3],
                              const vcgs_images* outs, int flags, void* stream);

/* Backward of the last vcgs_render_batch_forward of ctx.  g, views (cameras
 * and poses) and flags must be those of that forward (VCGS_E_INVALID
 * otherwise).  dl_dcolor, dl_ddepth, dl_dalpha: HOST arrays of n_views device
 * pointers to each view's upstream gradient ([3][H][W], [H][W], [H][W]); an
 * array or an entry may be NULL (zero).  grads (device, Gaussian shapes, any
 * field NULL) are OVERWRITTEN with dL/d(mean, scale, quat, opacity, color)
 * summed over the views (per view with VCGS_BATCH_PER_VIEW), dl_dpose (device
 * float [n_views][6] or NULL) with each view's pose gradient, as in
 * vcgs_render_backward.  With VCGS_BATCH_GRAPH the backward is captured into
 * its own hipGraph the first time (and again when a pointer argument
 * changes) and replayed. */
int vcgs_render_batch_backward(vcgs_ctx* ctx, const vcgs_gaussians* g, const vcgs_views* views,
                               const float* const* dl_dcolor, const float* const* dl_ddepth,
                               const float* const* dl_dalpha, vcgs_gaussian_buffers* grads, float* dl_dpose,
                               int flags, void* stream);

/* vcgs_render_batch that also adds, for every Gaussian, the number of pixels
 * of all the window's views whose composite blends it to hits [n] (device
 * uint32, accumulated as in vcgs_render_forward_hits: the mask step's hit
 * counts of a keyframe window in one pass, paper Sec. 3.3 eq. (13)).  A
 * captured graph adds them again on every replay. */
int vcgs_render_batch_hits(vcgs_ctx* ctx, const vcgs_gaussians* g, const vcgs_views* views, const float bg[3],
                           const float* const* target_color, const float* const* target_depth, float w_depth,
                           const vcgs_images* outs, vcgs_gaussian_buffers* grads, float* dl_dpose, float* loss,
                           int flags, uint32_t* hits, void* stream);

/* Waits for the last batched pass of ctx to finish.  Returns VCGS_OK, or
 * VCGS_E_CAPACITY if the pair buffers of that plan overflowed in any pass
 * since the previous check (those passes' results are incomplete; the
 * required pair count is then also readable with vcgs_last_required_pairs,
 * and the flag is cleared).  pairs (optional) receives the last pass's pair
 * count. */
int vcgs_batch_check(vcgs_ctx* ctx, int64_t* pairs);

/* After VCGS_E_CAPACITY: the pair count the overflowing pass needed (0 before
 * any overflow).  The next pass with that plan sizes its buffers for it. */
int64_t vcgs_last_required_pairs(const vcgs_ctx* ctx);

/* Camera centres x_c = -R^T t of n_views world-to-camera poses (HOST arrays;
 * centres [n_views][3]), the camera input of the view-dependent decode (paper
 * eq. (9)); evaluated in binary64 and rounded to binary32. */
void vcgs_camera_centres(int n_views, const vcgs_pose* poses, float* centres);

/* ---- serving: continuous batching of novel-view requests --------------- */

/* A server renders forward-only novel views of one HBM-resident map (the
 * paper's rendering of a reconstructed scene from new poses, Sec. 3.1 eqs.
 * (1)-(6)), batching the requests that are waiting into passes of up to
 * max_views views.  It has `slots` passes in flight at once, each on its own
 * stream (default priority) with its own buffers, so a pass that is admitted
 * while others run overlaps with them on the device.
 *
 * Admission is by sort-buffer memory: each slot holds pair buffers of
 * pair_budget (tile, Gaussian) pairs (16 bytes each plus the sort histograms);
 * a request is estimated at pixels * pairs_per_pixel pairs and a pass takes
 * waiting requests in arrival order while their estimates fit.  The estimate
 * starts at cfg->pairs_per_pixel and then follows 1.25 x the largest pairs per
 * pixel observed over the last 32 passes.  A pass whose actual pair count
 * exceeds its buffers is run again (its slot grown to the count, the estimate
 * raised); results never depend on the batching: every
 * request's images equal those of vcgs_render_forward of it alone, bit for
 * bit. */
typedef struct vcgs_server vcgs_server;
typedef struct {
    int32_t max_views;      /* 1..16 */
    int32_t slots;          /* passes in flight, 1..8 */
    int64_t pair_budget;    /* pairs per slot, > 0 */
    float pairs_per_pixel;  /* initial estimate, > 0 */
    float bg[3];
} vcgs_server_config;

/* The map's attribute pointers are kept (not copied) and must stay valid and
 * unchanged while the server lives.  Allocates all slot buffers up front
 * (about 104 bytes per Gaussian per view of max_views, plus the pair buffers,
 * per slot); VCGS_E_NOMEM if they do not fit. */
int vcgs_server_create(vcgs_ctx* ctx, const vcgs_gaussians* map, const vcgs_server_config* cfg,
                       vcgs_server** out);
/* Waits for every pass in flight, then frees the server's buffers. */
void vcgs_server_destroy(vcgs_server* srv);
/* Queues one request.  out: device images of the camera's size, written when
 * the request completes; they must stay valid until then.  The request's pass
 * runs after the work enqueued on `stream` so far (e.g. the map upload or the
 * last use of the output memory).  ticket receives the request's id (0, 1,
 * 2, ... in submission order).  Does not launch work.  Requests still queued
 * when the server is destroyed are dropped. */
int vcgs_server_submit(vcgs_server* srv, const vcgs_camera* cam, const vcgs_pose* pose, const vcgs_images* out,
                       int64_t* ticket, void* stream);
/* Collects passes that finished (their tickets into done[0 .. *n_done), at most
 * max_done; the rest are reported by later calls), then launches waiting
 * requests into free slots.  If nothing finished and nothing was launched it
 * polls again for up to timeout_us microseconds. */
int vcgs_server_progress(vcgs_server* srv, int64_t timeout_us, int64_t* done, int32_t max_done, int32_t* n_done);
/* Counters: requests queued, passes in flight, passes run, passes rerun after
 * an overflow, current pairs-per-pixel estimate. */
typedef struct {
    int64_t queued, in_flight, passes, reruns;
    float pairs_per_pixel;
} vcgs_server_stats;
int vcgs_server_stats_read(const vcgs_server* srv, vcgs_server_stats* out);

/* ---- mask training step (paper Sec. 3.3, eq. (13)) --------------------- */

/* vcgs_render_forward that also adds, for every Gaussian, the number of
 * pixels whose composite blends it (alpha >= 1/255, before the pixel stops)
 * to hits [n] (device uint32; accumulated, so a sliding window sums its
 * views; the caller zeroes it). */
int vcgs_render_forward_hits(vcgs_ctx* ctx, const vcgs_gaussians* g, const vcgs_camera* cam, const vcgs_pose* pose,
                             const float bg[3], vcgs_images* out, vcgs_state** state_out, uint32_t* hits,
                             void* stream);

/* Mask loss restricted to the view frustum: L_m = weight * mean over the
 * Gaussians with in_frustum_count[g] > 0 (e.g. the tile counts of a render
 * state; NULL = all n) of sigmoid(mask_logit[g]).  loss (device, 1 float, or
 * NULL) is overwritten; dl_dm (device [n] or NULL) gets weight * sigmoid'(m) /
 * N ADDED for the Gaussians in the frustum (others unchanged).  Deterministic. */
int vcgs_mask_loss(vcgs_ctx* ctx, int64_t n, const float* mask_logit, const uint32_t* in_frustum_count,
                   float weight, float* dl_dm, float* loss, void* stream);

/* Pruning at the end of a window: keep[g] = sigmoid(mask_logit[g]) > mask_eps
 * and hits[g] >= min_hits (hits NULL: the mask alone); kept_index receives the
 * kept Gaussians' indices in increasing order (capacity n; NULL to skip).
 * keep is uint8 [n] (or NULL).  *n_kept (host) receives their number; the call
 * synchronises the stream to read it. */
int vcgs_mask_prune(vcgs_ctx* ctx, int64_t n, const float* mask_logit, float mask_eps, const uint32_t* hits,
                    uint32_t min_hits, uint8_t* keep, uint32_t* kept_index, int64_t* n_kept, void* stream);

/* ---- tracking and bundle-adjustment losses (paper Sec. 3.5) ----------- */

/* Silhouette-masked colour + depth loss of eqs. (19) and (21):
 *   L = sum_p [S(p) > sil_thresh] (l_c(p) + lam_d l_d(p)),
 *   l_c(p) = sum_c e(C - C*) / (W H),  l_d(p) = e(D - D*) / |R| for D*(p) > 0,
 * |R| the number of pixels with a depth observation (D* > 0), e(x) = x^2
 * (norm 2, the paper's form) or |x| (norm 1).  img->alpha is the rendered
 * silhouette S.  dl_dcolor [3][H][W] and dl_ddepth [H][W] (device, both or
 * neither) are OVERWRITTEN with the gradient (0 where the mask is off);
 * loss (device float or NULL) is overwritten.  Deterministic. */
int vcgs_track_loss(vcgs_ctx* ctx, const vcgs_images* img, const float* target_color, const float* target_depth,
                    int32_t width, int32_t height, float lam_d, int32_t norm, float sil_thresh, float* dl_dcolor,
                    float* dl_ddepth, float* loss, void* stream);

/* ICP term of eq. (20), weighted: L = weight sum_i w_i |R p_i + t - q_i|^2.
 * p_i = mean [3][n] (device, world); q_i = nearest point of depth [H][W]
 * (device, the observed depth of the frame seen by cam, 0 = none) back-
 * projected at pixel centres, every stride-th pixel in each direction;
 * w_i = 1 iff |R p_i + t - q_i| < tau.  The association is held fixed.
 * loss (device float or NULL) overwritten; dmean [3][n] (device or NULL) and
 * dpose [6] (device or NULL; (rho, phi) of the left perturbation, as in
 * vcgs_render_backward) get the gradient ADDED; matched (device uint32 or NULL)
 * receives the number of Gaussians with w_i = 1.  Deterministic. */
int vcgs_icp_loss(vcgs_ctx* ctx, int64_t n, const float* mean, const vcgs_camera* cam, const vcgs_pose* pose,
                  const float* depth, float tau, int32_t stride, float weight, float* dmean, float* dpose,
                  float* loss, uint32_t* matched, void* stream);

/* SSIM term of bundle adjustment: L = weight (1 - mean SSIM(color, target))
 * over 3 channels and W H pixels (11 x 11 Gaussian window, sigma 1.5,
 * C1 = 0.01^2, C2 = 0.03^2, zero padding outside the image).  loss (device
 * float or NULL) overwritten; dl_dcolor [3][H][W] (device or NULL) gets
 * dL/dcolor ADDED (so it combines with vcgs_l1_loss or vcgs_track_loss). */
int vcgs_ssim_loss(vcgs_ctx* ctx, const float* color, const float* target_color, int32_t width, int32_t height,
                   float weight, float* dl_dcolor, float* loss, void* stream);

/* ---- residual vector quantization (paper Sec. 3.4, eqs. (14)-(15)) ---- */

/* L cascaded codebooks of P codes of dimension D: books is device float
 * [L][P][D] (row-major).  Limits: 1 <= D <= 32, 1 <= L <= 8, 1 <= P <= 256;
 * with a code gradient also L * P * ((D + 1) | 1) <= 16384. */
typedef struct {
    int32_t dim;
    int32_t stages;
    int32_t codes;
    const float* books;
} vcgs_rvq_books;

/* Assign n vectors x (device float [n][D], finite) stage by stage: stage l
 * picks the code of books[l] nearest to the residual x - xhat, xhat being the
 * sum of the codes picked so far (eq. (14)).  The distance is decided in
 * binary32 as |c|^2 - 2 c.r in a fixed order; ties go to the lowest index.
 * Outputs (each NULL to skip, all device):
 *   idx    [L][n], idx_bytes = 1 (uint8, P <= 256) or 4 (int32);
 *   recon  float [n][D]: xhat after the last stage;
 *   loss   1 float, overwritten: eq. (15), 1/(n P) sum over stages and vectors
 *          of |r - C[i]|^2;
 *   dbooks float [L][P][D]: the loss's gradient to the codes is ADDED (the
 *          residual is under a stop-gradient, so x gets none).
 * Code sums inside a block are exact 64-bit fixed point (2^-32 units; a
 * block's sum of one residual component must stay below 2^31 in magnitude),
 * so every output, dbooks included, is bit-reproducible; idx and recon are
 * exact. */
int vcgs_rvq_assign(vcgs_ctx* ctx, const vcgs_rvq_books* q, int64_t n, const float* x, void* idx, int32_t idx_bytes,
                    float* recon, float* loss, float* dbooks, void* stream);

/* ---- anchor decode ---------------------------------------------------- */

/* Voxel anchors (paper Sec. 3.2): position x_a [3][na], feature f_a
 * [na][feat_dim] (row-major), scaling l [3][na], offsets O [na][k][3]. */
typedef struct {
    int64_t n_anchor;
    int32_t k;
    int32_t feat_dim;   /* must be 32 */
    const float* xa;
    const float* feat;
    const float* scaling;
    const float* offset;
} vcgs_anchors;

/* Decoder MLP: h = ReLU(W1 f + b1), y = W2 h + b2.  W1 [32][32], b1 [32],
 * W2 [k*11][32], b2 [k*11] (row-major, out x in).  Per offset i the 11 outputs
 * y[11 i ..] are [opacity, r, g, b, 3 log-scales, quaternion w, x, y, z]. */
typedef struct {
    const float* W1;
    const float* b1;
    const float* W2;
    const float* b2;
} vcgs_mlp;

/* Residual codebook (paper Sec. 3.4, eq. (14) first line): value of Gaussian
 * j = sum over stages s of books[s][idx[s][j]][0..6] = (3 log-scales,
 * quaternion).  books [stages][size][7], idx int32 [stages][na*k]; an index
 * outside [0, size) is clamped into it. */
typedef struct {
    int32_t stages;
    int32_t size;
    const float* books;
    const int32_t* idx;
} vcgs_codebook;

/* Decode anchors into na*k Gaussians (Gaussian index a*k + i), paper eqs. (7)-(8):
 *   mean = x_a + O_i * l (element-wise), opacity = sigmoid, colour = sigmoid,
 *   scale = exp(log-scale), quaternion passed on raw.
 *   If cb is non-NULL, log-scale and quaternion come from the codebook instead
 *   of the MLP.  If mask_logit [na*k] is non-NULL, Gaussians with
 *   sigmoid(m) <= mask_eps get opacity 0 and scale 0 (paper eqs. (11)-(12)),
 *   which the renderer culls.
 *   out: device buffers of na*k Gaussians, overwritten.
 *   Limits: feat_dim = 32, hidden = 32, 1 <= k <= 16. */
int vcgs_decode_anchors(vcgs_ctx* ctx, const vcgs_anchors* a, const vcgs_mlp* mlp,
                        const vcgs_codebook* cb, const float* mask_logit, float mask_eps,
                        vcgs_gaussian_buffers* out, void* stream);

/* Gradients of the decode.  Every output pointer may be NULL (not computed);
 * all are OVERWRITTEN, with the shapes of the matching input. */
typedef struct {
    float* feat;
    float* offset;
    float* scaling;
    float* xa;
    float* W1;
    float* b1;
    float* W2;
    float* b2;
    float* books;       /* [stages][size][7]: straight-through sums over the Gaussians using each row */
    float* mask_logit;  /* [na*k]: sigmoid'(m) (s . dL/ds_hat + alpha dL/dalpha_hat); 0 when pruned */
    float* cam;         /* [3]: dL/d camera centre (view-dependent decode only; ignored otherwise) */
} vcgs_anchor_grads;

/* dG: dL/d(decoded Gaussians) (device, na*k Gaussians, e.g. from
 * vcgs_render_backward).  Same a, mlp, cb, mask_logit, mask_eps as the forward. */
int vcgs_decode_anchors_backward(vcgs_ctx* ctx, const vcgs_anchors* a, const vcgs_mlp* mlp,
                                 const vcgs_codebook* cb, const float* mask_logit, float mask_eps,
                                 const vcgs_gaussian_buffers* dG, vcgs_anchor_grads* out, void* stream);

/* View-dependent decode, paper eqs. (8)-(9): the MLP input is the 36-d
 * [f_a, delta, d] with delta = |x_a - x_c| and d = (x_a - x_c) / delta for the
 * camera centre x_c = cam_centre (host, 3 floats; for a world-to-camera pose
 * {R|t} it is -R^T t).  mlp->W1 is [32][36] (row-major, the last four columns
 * weigh delta, d_x, d_y, d_z); everything else as vcgs_decode_anchors.  An
 * anchor at the camera centre (delta = 0) has no direction: such input is
 * outside the operation's domain. */
int vcgs_decode_anchors_view(vcgs_ctx* ctx, const vcgs_anchors* a, const vcgs_mlp* mlp, const vcgs_codebook* cb,
                             const float* mask_logit, float mask_eps, const float cam_centre[3],
                             vcgs_gaussian_buffers* out, void* stream);

/* Gradients of vcgs_decode_anchors_view: as vcgs_decode_anchors_backward, with
 * W1 [32][36], xa including the path through delta and d, and out->cam (if
 * non-NULL) receiving dL/d(camera centre).  For the left-perturbed pose the
 * centre moves by -R^T rho, so its share of dL/dxi is (-R dL/dcam, 0). */
int vcgs_decode_anchors_view_backward(vcgs_ctx* ctx, const vcgs_anchors* a, const vcgs_mlp* mlp,
                                      const vcgs_codebook* cb, const float* mask_logit, float mask_eps,
                                      const float cam_centre[3], const vcgs_gaussian_buffers* dG,
                                      vcgs_anchor_grads* out, void* stream);

/* The view-dependent decode (paper eqs. (8)-(9)) for n_views camera centres
 * in one launch, e.g. the keyframes of a bundle-adjustment window (Sec. 3.5).
 * cam_centres: host, [n_views][3]; 1 <= n_views <= VCGS_DECODE_MAX_VIEWS.
 * View v's Gaussians are written to block v of a stacked per-view set: out
 * arrays hold n_views * na*k Gaussians, each view an ordinary SoA set
 * (mean [V][3][na*k], quat [V][4][na*k], opacity [V][na*k], ...), the layout
 * that vcgs_render_batch reads with VCGS_BATCH_PER_VIEW.  Each view's block
 * equals vcgs_decode_anchors_view for that centre, bit for bit. */
#define VCGS_DECODE_MAX_VIEWS 16
int vcgs_decode_anchors_views(vcgs_ctx* ctx, const vcgs_anchors* a, const vcgs_mlp* mlp, const vcgs_codebook* cb,
                              const float* mask_logit, float mask_eps, int n_views, const float* cam_centres,
                              vcgs_gaussian_buffers* out, void* stream);

/* Gradients of vcgs_decode_anchors_views: dG stacked per view as above.  The
 * anchor, MLP, codebook and mask gradients in out are the sums over the views
 * (one launch, deterministic); out->cam (if non-NULL) receives dL/d(camera
 * centre) per view, [n_views][3]. */
int vcgs_decode_anchors_views_backward(vcgs_ctx* ctx, const vcgs_anchors* a, const vcgs_mlp* mlp,
                                       const vcgs_codebook* cb, const float* mask_logit, float mask_eps,
                                       int n_views, const float* cam_centres, const vcgs_gaussian_buffers* dG,
                                       vcgs_anchor_grads* out, void* stream);

/* The pose's share of the camera-centre input of the view-dependent decode
 * (paper eq. (9)): for a world-to-camera pose {R|t} the centre -R^T t moves by
 * -R^T rho under the left perturbation, so dpose[v] (device, 6 floats per
 * view: rho, phi) gets -R_v dcam[v] ADDED to its rho part (phi unchanged).
 * poses: host, n_views of them (R is passed with the launch, no copy);
 * dcam: device [n_views][3], e.g. out->cam of the decode backward.
 * 0 <= n_views <= VCGS_DECODE_MAX_VIEWS. */
int vcgs_centre_pose_grad(vcgs_ctx* ctx, int n_views, const vcgs_pose* poses, const float* dcam, float* dpose,
                          void* stream);

/* A novel-view server (vcgs_server_create) over the view-dependent decode of
 * anchors (paper eqs. (8)-(9)):
 * every pass decodes its requests' camera centres in one launch (as
 * vcgs_decode_anchors_views; x_c = -R^T t computed in binary64 from the
 * pose's values and rounded to binary32) into the slot's per-view sets, then
 * renders each request from its own set.  A request's images equal
 * vcgs_render_forward of vcgs_decode_anchors_view at that centre, bit for bit.
 * a, mlp (W1 [32][36]), cb and mask_logit are kept (not copied) and must stay
 * valid and unchanged while the server lives.  Per slot it adds 56 bytes per
 * Gaussian per view of max_views for the decoded sets. */
int vcgs_server_create_anchors(vcgs_ctx* ctx, const vcgs_anchors* a, const vcgs_mlp* mlp, const vcgs_codebook* cb,
                               const float* mask_logit, float mask_eps, const vcgs_server_config* cfg,
                               vcgs_server** out);

/* ---- kernel configuration ---------------------------------------------- */

/* Process-wide settings read by every later launch (all contexts):
 *   VCGS_OPT_PPL_FWD / VCGS_OPT_PPL_BWD: pixels per lane of the forward /
 *     backward compositing, 1, 2 or 4 (a 16x16 tile is walked by 4, 2 or 1 waves);
 *   VCGS_OPT_CULL: 1 = skip, per wave, tile-list entries whose 1/255 ellipse
 *     misses the wave's pixels (results are identical either way), 0 = visit all;
 *   VCGS_OPT_SCHED: order in which compositing blocks take tiles, 0 = linear
 *     (default), 1 = XCD-aware (each of the 8 XCDs gets a contiguous run of
 *     tiles, so that neighbouring tiles share its L2); results are identical
 *     either way;
 *   VCGS_OPT_BWD_MERGE: with 1 pixel per lane in the backward, 1 = the four
 *     waves of a tile step through its list together and merge their
 *     per-Gaussian sums in LDS before adding them to the gradient (one atomic
 *     per value per tile instead of per quarter tile), 0 = independent waves
 *     (default); equal up to the order of floating-point sums.
 * Defaults: 1 pixel per lane both ways, culling on, linear order, no merging.
 * A captured batch graph keeps the settings it was captured with.
 * Invalid keys or values return VCGS_E_INVALID and change nothing. */
enum { VCGS_OPT_PPL_FWD = 1, VCGS_OPT_PPL_BWD = 2, VCGS_OPT_CULL = 3, VCGS_OPT_SCHED = 4, VCGS_OPT_BWD_MERGE = 5 };
int vcgs_set_option(int key, int value);
int vcgs_get_option(int key, int* value);

/* ---- stage timing ------------------------------------------------------ */

/* Stages timed with HIP events on the caller's stream when profiling is on. */
enum {
    VCGS_STAGE_DECODE = 0,        /* anchor decode (MFMA MLP, codebook, mask) */
    VCGS_STAGE_PREPROCESS = 1,    /* EWA projection, keys, tile rectangles */
    VCGS_STAGE_DEPTH_SORT = 2,    /* radix sort of the depth keys */
    VCGS_STAGE_PAIR_SCAN = 3,     /* pair counts in depth order, their scan */
    VCGS_STAGE_EMIT = 4,          /* (tile, Gaussian) pair emission */
    VCGS_STAGE_TILE_SORT = 5,     /* stable radix sort of the pairs by tile */
    VCGS_STAGE_TILE_RANGES = 6,   /* per-tile [start, end) */
    VCGS_STAGE_COMPOSITE = 7,     /* forward compositing */
    VCGS_STAGE_LOSS = 8,          /* L1 loss and its image gradients */
    VCGS_STAGE_COMPOSITE_BWD = 9, /* replayed compositing adjoint */
    VCGS_STAGE_PREPROCESS_BWD = 10, /* projection adjoint and pose reduction */
    VCGS_STAGE_DECODE_BWD = 11,   /* decode adjoint (MFMA) */
    VCGS_STAGE_COUNT = 16
};

/* Turn per-stage event timing on (1) or off (0); turning it on clears the totals. */
int vcgs_profile_enable(vcgs_ctx* ctx, int on);
/* Stages that event timing covers while on: bit s = VCGS_STAGE s (default all).
 * Each timed stage records two events per launch on the stream, which shows in
 * the time between kernels; timing one stage keeps that cost to two events. */
int vcgs_profile_stages(vcgs_ctx* ctx, uint32_t mask);
/* Synchronises the recorded events and returns the summed duration (ms) and
 * the number of timed launches of `stage` since profiling was enabled. */
int vcgs_profile_read(vcgs_ctx* ctx, int stage, double* total_ms, int64_t* launches);

/* Work counters of the last forward and backward compositing call, filled
 * when counting is on (slower; for measurement only):
 *   fwd_evals   (pixel, list entry) footprint evaluations in the forward
 *   fwd_blends  of which blended into the pixel
 *   bwd_evals   footprint evaluations replayed in the backward
 *   bwd_blends  of which produced gradients
 *   bwd_atomics per-Gaussian gradient flushes (10 atomics each) */
int vcgs_count_enable(vcgs_ctx* ctx, int on);
int vcgs_count_read(vcgs_ctx* ctx, int64_t out[5]);

#ifdef __cplusplus
}
#endif
#endif /* VCGS_H */
