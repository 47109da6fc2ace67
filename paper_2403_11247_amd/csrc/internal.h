// Internal declarations of the vcgs HIP library (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <algorithm>
#include <stdint.h>

#include "../../include/vcgs.h"

namespace vcgs {

// Footprint and stop rule thresholds (FP32 constants; see the renderer notes
// in render.hip).
constexpr float kAlphaMin = 1.0f / 255.0f;
constexpr float kAlphaMax = 0.99f;
constexpr float kTMin = 1e-4f;
constexpr float kLowPass = 0.3f;
constexpr float kLowPass2 = 0.09f;
constexpr float kHalfLog2e = 0.72134752f;      // 1 / (2 ln 2)
constexpr float kLn2 = 0.69314718f;
constexpr float kClampFov = 1.3f;
constexpr float kTwoLn2 = 1.3862944f;
constexpr int kTile = 16;
constexpr int kMaxViews = 16;  // views rendered by one batched call

// Camera as passed to kernels.
struct CamK {
    int W, H;
    float fx, fy, cx, cy, znear;
    int tiles_x, tiles_y;
    float limx, limy;
    uint32_t tile_base;  // first global tile id of this view
};
struct PoseK {
    float R[9];
    float t[3];
};

// Per-view tables passed by value.  Entry e of the projection outputs is
// (view e / n, Gaussian e % n); global tile ids are view-major.
struct ProjTab {
    int n_views;
    int per_view;  // 0: one Gaussian set for all views; 1: view v reads its own set [v*n, (v+1)*n)
    int64_t n;     // Gaussians per view
    CamK cam[kMaxViews];
    PoseK pose[kMaxViews];
};
struct ViewTab {
    int n_views;
    int64_t n;
    uint32_t tile_end[kMaxViews];  // exclusive end of each view's global tile ids
    CamK cam[kMaxViews];
    float* color[kMaxViews];
    float* depth[kMaxViews];
    float* alpha[kMaxViews];
    float* t_final[kMaxViews];
    uint32_t* n_contrib[kMaxViews];
    const float* dl_dc[kMaxViews];
    const float* dl_dd[kMaxViews];
    const float* dl_da[kMaxViews];
    float bg[3];
    uint32_t* hits;  // optional: per-Gaussian count of blended pixels, accumulated (Gaussian = entry % n)
    // optional: host-visible pinned words that receive flags_src[0..1] (the
    // pass's pair count and overflow word) from the forward's first thread,
    // so that a poller needs no copy after the pass
    uint32_t* flags_out;
    const uint32_t* flags_src;
};

// Projected splat record, 64 bytes: (u, v, u_lo, v_lo) (s1 ex, s1 ey, s2 ex, s2 ey)
// (o, r, g, b) (depth, s1, s2, -).  The screen position is u + u_lo (a binary32 pair),
// (ex, ey) the unit eigenvector of the larger eigenvalue lambda1 of Sigma' + 0.3 I and
// s = sqrt(1 / (2 ln2 lambda)) for each eigenvalue.  The footprint exponent in base 2 is
// -(q1^2 + q2^2) with q1 = s1 d . (ex, ey), q2 = s2 d . (-ey, ex), d = pixel centre - (u, v).
struct Splat {
    float4 a, b, c, d;
};

// Per-entry gradient sums of the compositing adjoint, 12 floats: five sums of
// dL/dpower against the scaled pixel offset (q1, q2) in the footprint's eigen
// frame (q1, q2, q1^2, q1 q2, q2^2; the projection adjoint unscales and rotates
// them into dL/d(u, v) and dL/d(conic)), dopacity, dr, dg, db, ddepth, -, -.
constexpr int kG2 = 12;

CamK make_camk(const vcgs_camera& c, uint32_t tile_base = 0);
PoseK make_posek(const vcgs_pose& p);

// Element counts that may live on the device: when dev != nullptr the count is
// min(*dev, cap), otherwise cap.  Grids are sized from cap.
struct Count {
    int64_t cap;
    const uint32_t* dev;
};

// ---- launchers (all asynchronous on `s`) --------------------------------
// preprocess.hip
// The backward reads the table from device memory (t_dev) so that a captured
// graph can be replayed with new poses.  The projection reads it from t_dev
// too, unless by_value: then it takes t as a kernel argument (no upload) and
// writes the copy at t_dev (when non-null) for the backward.
// g2_zero (optional): kG2 floats per entry, zeroed for every visible entry.
struct ZeroSegs;
// zero: words the pass needs at zero (the projection's threads clear them too), or null.
void launch_preprocess(const ProjTab& t, ProjTab* t_dev, const vcgs_gaussians& g, Splat* rec,
                       uint32_t* depth_key, uint2* rect, uint32_t* count, float* g2_zero, hipStream_t s,
                       const ZeroSegs* zero = nullptr, bool by_value = false);
int preprocess_bwd_blocks(int64_t n);
// g2, count and rec have n_views * n entries; pose_partial holds n_views * blocks * 6 floats.
void launch_preprocess_bwd(const ProjTab& t, const ProjTab* t_dev, const vcgs_gaussians& g, const uint32_t* count,
                           const Splat* rec, const float* g2, const vcgs_gaussian_buffers& out, float* pose_partial,
                           int blocks, hipStream_t s);
// dl_dpose: n_views * 6 floats
void launch_pose_reduce(const float* partial, int n_views, int nblocks, float* dl_dpose, hipStream_t s);

// sort.hip
struct SortTemp {
    uint32_t* keys_alt;
    uint32_t* vals_alt;
    uint32_t* head;     // sort_head_words(): digit counts and partition counters, zero on entry
    uint32_t* state;    // sort_state_words(cap): look-back state (the sort zeroes what it uses)
    int64_t state_words = 0;  // words at state if more than sort_state_words(cap) (0: exactly that)
};
constexpr int64_t kMaxSortItems = (1ll << 30) - 1;
int radix_blocks(int64_t n);
int64_t sort_head_words();
int64_t sort_state_words(int64_t cap);
int64_t scan_temp_words(int64_t n);
// Stable LSD radix sort of (keys, vals) on bits [0, end_bit), end_bit <= 32.
// t.head must be zero on entry (launch_zero_u32 clears it with other buffers
// in one launch).  With identity_vals the input values are 0..n-1 and `vals`
// is not read (it must still hold cap entries).  Returns 0 if the result is in (keys, vals), 1 if
// it is in (t.keys_alt, t.vals_alt).  At most kMaxSortItems items (returns -1
// and does nothing above that).
// With kept != nullptr, items whose key is kDropKey are dropped (the others
// keep their order) and *kept receives a device pointer to the number kept.
// With keys_src, the first pass reads its keys from there (not modified) and
// `keys` is only used as a buffer.
constexpr uint32_t kDropKey = 0xFFFFFFFFu;
// size_hint (> 0): the expected item count when the capacity n.cap is a
// generous bound; the partition size follows it if t.state holds enough words,
// and the passes' grids are sized for it (with a margin; any count up to the
// capacity is still sorted).
int radix_sort_u32(uint32_t* keys, uint32_t* vals, bool identity_vals, Count n, int end_bit, const SortTemp& t,
                   hipStream_t s, const uint32_t** kept = nullptr, const uint32_t* keys_src = nullptr,
                   int64_t size_hint = 0, bool hist_done = false);
// What a kernel that writes the keys must do so that radix_sort_u32 can skip
// its histogram launch (hist_done, no dropping; same n, end_bit, t and
// size_hint): add each key's digit of pass p, (key >> 8p) & 255 for p <
// passes, to ghist[(b % kSortHistCopies) * kSortPassStride + p * 256 + digit]
// (any copy b; t.head is zero on entry), and zero, for every pass p, the
// ceil(items / part_items) * 256 words at state + p * state_stride, items
// being the device count.  ghist == nullptr: nothing to do (n.cap <= 0).
constexpr int kSortHistCopies = 8;
constexpr int kSortPassStride = 4 * 256;
struct SortPrep {
    uint32_t* ghist = nullptr;
    uint32_t* state = nullptr;
    int64_t state_stride = 0, part_items = 0;
    int passes = 0;
};
SortPrep radix_sort_prep(Count n, int end_bit, const SortTemp& t, int64_t size_hint = 0);
// Exclusive scan of n uint32 values (out may equal in); if total != nullptr
// the sum is written there.  Sums saturate at 2^31 instead of wrapping.
void exclusive_scan_u32(const uint32_t* in, uint32_t* out, int64_t n, uint32_t* total, uint32_t* tmp,
                        hipStream_t s);
// Words of pair_offsets' look-back state for n entries (zero before each call).
int64_t pair_scan_words(int64_t n);
// Tile counts of the depth-ordered entries and their exclusive prefix sums in
// one launch: cnt[k] = count[order[k]] for k below the device count n.dev
// (0 up to n.cap), offs[k] = sum of cnt[j] for j < k, *total = the sum (all
// saturating at 2^31).  state: pair_scan_words(n.cap) words, zero on entry.
// host_total (optional): pinned host word that also receives the sum, so that
// a caller that synchronises needs no copy.
void pair_offsets(const uint32_t* order, const uint32_t* count, Count n, uint32_t* cnt, uint32_t* offs,
                  uint32_t* total, uint32_t* state, hipStream_t s, uint32_t* host_total = nullptr);

// binning.hip
struct EmitTab {
    int n_views;
    int64_t n;  // entries per view
    int tiles_x[kMaxViews];
    uint32_t tile_base[kMaxViews];
};
// out[k] = count[order[k]] for k < min(n, *nvis), 0 above (order is only read below *nvis).
// Entries k < min(n_entries, *nvis) of the depth order (offsets offs and
// counts cnt in that order) emit their pairs; writes pairs p < cap only; if the
// total exceeds cap raises *overflow to the total (when non-null; the flag
// keeps the largest such total until the host clears it).  chunk_start: scratch
// of emit_chunk_words(cap) words.
// With sp.ghist set, it also does what sp asks of the tile ids for the tile
// sort (see radix_sort_prep); returns false if it launched nothing (then the
// sort must build its own histogram).
// grid_items (> 0): the expected pair count when cap is a generous bound; the
// grid is sized for it (any count up to cap is still emitted).
bool launch_emit_pairs(const EmitTab& t, int64_t n_entries, const uint32_t* nvis, const uint32_t* order,
                       const uint32_t* offs, const uint32_t* cnt, const uint2* rect, uint32_t* chunk_start,
                       uint32_t* tile_ids, uint32_t* gids, int64_t cap, const uint32_t* total, uint32_t* overflow,
                       const SortPrep& sp, hipStream_t s, int64_t grid_items = 0);
int64_t emit_chunk_words(int64_t cap);
void launch_tile_ranges(Count P, const uint32_t* tile_sorted, uint32_t n_tiles, uint32_t* ranges, hipStream_t s,
                        int64_t grid_items = 0);
void launch_fill_u32(uint32_t* p, uint32_t v, int64_t n, hipStream_t s);
// Zeroes up to four buffers (null or empty ones are skipped) in one launch.
constexpr int kZeroSegs = 5;
struct ZeroSegs {
    uint32_t* p[kZeroSegs];
    int64_t n[kZeroSegs];
};
// Drops null or empty segments and returns the total word count.
inline int64_t zero_segs_normalise(ZeroSegs& z)
{
    int64_t total = 0;
    for (int i = 0; i < kZeroSegs; ++i) {
        if (!z.p[i] || z.n[i] < 0) z.n[i] = 0;
        total += z.n[i];
    }
    return total;
}
// Zeroes words [0, total) of the segments, thread tid of nthreads taking every
// nthreads-th word (a normalised z).
__device__ __forceinline__ void zero_segs(const ZeroSegs& z, int64_t total, int64_t tid, int64_t nthreads)
{
    for (int64_t i = tid; i < total; i += nthreads) {
        int64_t k = i;
        int seg = 0;
        while (seg < kZeroSegs - 1 && k >= z.n[seg]) {
            k -= z.n[seg];
            ++seg;
        }
        z.p[seg][k] = 0u;
    }
}

// Sums of N per-thread values over a 256-thread block in a fixed order
// (butterfly within each wave, then the four waves in order): the results are
// in thread 0.  lds: 4 * N doubles of shared memory.  Every thread of the
// block must call it.
template <int N>
__device__ __forceinline__ void block_sum_f64(double (&v)[N], double* lds)
{
#pragma unroll
    for (int i = 0; i < N; ++i)
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) v[i] += __shfl_xor(v[i], o, 64);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0)
#pragma unroll
        for (int i = 0; i < N; ++i) lds[w * N + i] = v[i];
    __syncthreads();
    if (threadIdx.x == 0)
#pragma unroll
        for (int i = 0; i < N; ++i) v[i] = (lds[i] + lds[N + i]) + (lds[2 * N + i] + lds[3 * N + i]);
}
void launch_zero_u32(const ZeroSegs& z, hipStream_t s);
void launch_fill_f32(float* p, float v, int64_t n, hipStream_t s);
void launch_copy_u32(uint32_t* dst, const uint32_t* src, Count n, hipStream_t s);

// render.hip
// counters (optional, 5 x u64): see vcgs_count_read.
void launch_composite_fwd(const ViewTab& v, uint32_t total_tiles, const Splat* rec, const uint32_t* gids,
                          const uint32_t* ranges, unsigned long long* counters, hipStream_t s);
void launch_composite_bwd(const ViewTab& v, uint32_t total_tiles, const Splat* rec, const uint32_t* gids,
                          const uint32_t* ranges, float* g2, unsigned long long* counters, hipStream_t s);
int l1_loss_blocks(int64_t npix);
// Per-view L1 losses of a batch; view v owns loss blocks [block0[v], block0[v+1]),
// block0[v+1] - block0[v] = l1_loss_blocks(npix[v]).
struct LossTab {
    int n_views;
    float w_depth;
    int64_t npix[kMaxViews];
    int block0[kMaxViews + 1];
    const float* c[kMaxViews];
    const float* d[kMaxViews];
    const float* tc[kMaxViews];
    const float* td[kMaxViews];
    float* dlc[kMaxViews];
    float* dld[kMaxViews];
};
// loss: n_views floats (or null); partial: block0[n_views] floats of scratch.
void launch_l1_loss_views(const LossTab& t, float* loss, float* partial, hipStream_t s);
// partial: l1_loss_blocks(npix) floats of scratch (only used when loss != nullptr)
void launch_l1_loss(int64_t npix, const float* c, const float* d, const float* tc, const float* td,
                    float w_depth, float* dl_dc, float* dl_dd, float* loss, float* partial, hipStream_t s);

// mask.hip: mask loss over the view frustum and pruning (paper eq. (13)).
// in_frustum: per-Gaussian tile counts of the view (count > 0 = in the frustum).
// partial: mask_loss_blocks(n) * 2 floats of scratch.
int mask_loss_blocks(int64_t n);
void launch_mask_loss(int64_t n, const float* logit, const uint32_t* count, float weight, float* dl_dm, float* loss,
                      float* partial, hipStream_t s);
// keep[g] = sigmoid(m) > eps && hits[g] >= min_hits (m above thr = logit(eps));
// kept_index: stable compaction; n_kept (device, 1 word).  tmp: scan_temp_words(n) + 8 words.
void launch_mask_prune(int64_t n, const float* logit, float thr, const uint32_t* hits, uint32_t min_hits,
                       uint8_t* keep, uint32_t* flags_tmp, uint32_t* offs_tmp, uint32_t* kept_index,
                       uint32_t* n_kept, uint32_t* scan_tmp, hipStream_t s);

// Residual vector quantization (rvq.hip).  tab: L * P * (rvq_padded_dim(D) + 4)
// floats; partial: rvq_partial_floats(...) floats; red: rvq_red_doubles(...) doubles.
int rvq_padded_dim(int d);
int64_t rvq_partial_floats(int64_t n, int L, int P, int D, bool grad);
int64_t rvq_red_doubles(int64_t n, int L, int P, int D, bool grad);
// false: the device refused the LDS the launch needs (nothing was launched)
bool launch_rvq(int64_t n, int D, int L, int P, const float* books, const float* x, void* idx, int idx_bytes,
                float* recon, float* loss, float* dbooks, float* tab, float* partial, double* red, hipStream_t s);

// Tracking / BA losses (track.hip).
int64_t track_partial_floats(int W, int H);
void launch_track_loss(int W, int H, const float* C, const float* D, const float* A, const float* tC,
                       const float* tD, float lam_d, int norm, float thresh, float* dlc, float* dld, float* loss,
                       float* partial, hipStream_t s);
// dm: 9 * W * H floats; partial: ssim_partial_floats(W, H) floats
int64_t ssim_partial_floats(int W, int H);
void launch_ssim_loss(int W, int H, const float* X, const float* Y, float weight, float* dlc, float* loss, float* dm,
                      float* partial, hipStream_t s);
// partial: 8 * icp_blocks(n) floats (at least 8); tmin: icp_tile_floats(W, H) floats
int icp_blocks(int64_t n);
int64_t icp_tile_floats(int W, int H);
void launch_icp(int64_t n, const float* mean, const float* depth, int W, int H, float fx, float fy, float cx,
                float cy, const float R[9], const float t[3], float tau, int stride, float weight, float* dmean,
                float* loss, float* dpose, uint32_t* matched, float* partial, float* tmin, hipStream_t s);

// Process-wide kernel configuration (vcgs_set_option).
struct Options {
    int ppl_fwd = 1;  // pixels per lane of the forward compositing (1, 2, 4)
    int ppl_bwd = 1;  // pixels per lane of the backward compositing (1, 2, 4)
    int cull = 1;     // per-wave ellipse culling of tile-list entries
    int sched = 0;    // compositing block order: 0 linear, 1 XCD-aware (consecutive tiles on one XCD)
    int bwd_merge = 0;  // backward at 1 pixel per lane: a tile's 4 waves merge their totals before the atomics
};
Options& options();

// decode.hip
constexpr int kDecodeMaxViews = 16;  // camera centres per decode launch

struct DecodeArgs {
    int64_t na;
    int k;
    const float *xa, *feat, *scaling, *offset;
    const float *W1, *b1, *W2, *b2;
    int stages, cb_size;
    const float* books;
    const int32_t* idx;
    const float* mask_logit;
    float mask_thr;  // keep iff logit > mask_thr
    int in_dim;      // 32: feature input; 36: [feature, distance, direction] from the camera centres cam
    int views;       // number of camera centres (1 without the view input); outputs and dG are stacked per view
    float cam[kDecodeMaxViews][3];
};
// Validates the decode inputs and fills d.  cam: NULL, or `views` camera centres
// (host, [views][3]) for the view-dependent decode.
int make_decode_args(const vcgs_anchors* a, const vcgs_mlp* mlp, const vcgs_codebook* cb, const float* mask_logit,
                     float mask_eps, DecodeArgs* d, const float* cam = nullptr, int views = 1);
void launch_decode_fwd(const DecodeArgs& a, const vcgs_gaussian_buffers& out, hipStream_t s);
int decode_bwd_blocks(int64_t na, int k);
__host__ __device__ int64_t decode_bwd_partial_floats(int k, int in_dim, int views);
// dvbuf: na*k*8 floats and book_partial: books_grad_blocks(na*k) * stages * cb_size * 7
// floats of scratch for the codebook gradient (NULL: device atomics on the rows).
void launch_decode_bwd(const DecodeArgs& a, const vcgs_gaussian_buffers& dG, const vcgs_anchor_grads& out,
                       float* partial, int nblocks, float* dvbuf, float* book_partial, hipStream_t s);
int books_grad_blocks(int64_t n);
struct CentreTab {
    int views;
    float R[kDecodeMaxViews][9];  // world-to-camera rotations, row-major
};
// dpose [views][6] += (-R dL/dx_c, 0) for dcam [views][3] (device).
void launch_centre_pose_grad(const CentreTab& t, const float* dcam, float* dpose, hipStream_t s);
constexpr size_t kBookLdsMax = 150 * 1024;  // largest codebook stage table summed in LDS

}  // namespace vcgs
