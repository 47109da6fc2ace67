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
constexpr float kNegHalfLog2e = -0.72134752f;  // -1 / (2 ln 2)
constexpr float kLn2 = 0.69314718f;
constexpr float kClampFov = 1.3f;
constexpr float kTwoLn2 = 1.3862944f;
constexpr int kTile = 16;

// Camera and pose as passed to kernels (by value).
struct CamK {
    int W, H;
    float fx, fy, cx, cy, znear;
    int tiles_x, tiles_y;
    float limx, limy;
    uint32_t tile_base;  // added to every tile id (several views share one id space)
};
struct PoseK {
    float R[9];
    float t[3];
};

// Projected splat record, 64 bytes: (u, v, u_lo, v_lo) (ex, ey, j1, j2) (o, r, g, b) (depth, -, -, -).
// The screen position is u + u_lo (a binary32 pair).  The footprint exponent in base 2
// is j1 p1^2 + j2 p2^2 with p1 = d . (ex, ey), p2 = d . (-ey, ex), d = pixel centre -
// (u, v), j = -1 / (2 ln2 lambda) for the two eigenvalues of Sigma' + 0.3 I.
struct Splat {
    float4 a, b, c, d;
};

// Per-Gaussian gradient of the 2D quantities, 12 floats:
// du, dv, dA, dB, dC, dopacity, dr, dg, db, ddepth, -, -.
constexpr int kG2 = 12;

CamK make_camk(const vcgs_camera& c, uint32_t tile_base = 0);
PoseK make_posek(const vcgs_pose& p);

// ---- launchers (all asynchronous on `s`) --------------------------------
// preprocess.hip
void launch_preprocess(int64_t n, const vcgs_gaussians& g, const CamK& cam, const PoseK& pose,
                       Splat* rec, uint32_t* depth_key, uint2* rect, uint32_t* count, hipStream_t s);
void launch_preprocess_bwd(int64_t n, const vcgs_gaussians& g, const CamK& cam, const PoseK& pose,
                           const uint32_t* count, const float* g2, const vcgs_gaussian_buffers& out,
                           float* pose_partial, int pose_blocks, hipStream_t s);
int preprocess_bwd_blocks(int64_t n);
void launch_pose_reduce(const float* partial, int nblocks, float* dl_dpose, hipStream_t s);

// sort.hip
struct SortTemp {
    uint32_t* keys_alt;
    uint32_t* vals_alt;
    uint32_t* hist;     // >= 256 * radix_blocks(n)
    uint32_t* scan_tmp; // >= scan_temp_words(256 * radix_blocks(n))
};
int radix_blocks(int64_t n);
int64_t scan_temp_words(int64_t n);
// Stable LSD radix sort of (keys, vals) on bits [0, end_bit).  With
// identity_vals the input values are 0..n-1 and `vals` is not read (it must
// still hold n entries).  Returns 0 if the result is in (keys, vals), 1 if it
// is in (t.keys_alt, t.vals_alt).
int radix_sort_u32(uint32_t* keys, uint32_t* vals, bool identity_vals, int64_t n, int end_bit, const SortTemp& t,
                   hipStream_t s);
// Exclusive scan of n uint32 values (out may equal in); if total != nullptr
// the sum is written there.
void exclusive_scan_u32(const uint32_t* in, uint32_t* out, int64_t n, uint32_t* total, uint32_t* tmp,
                        hipStream_t s);

// binning.hip
void launch_gather_counts(int64_t n, const uint32_t* order, const uint32_t* count, uint32_t* out,
                          hipStream_t s);
void launch_emit_pairs(int64_t n, const uint32_t* order, const uint32_t* offs, const uint32_t* count,
                       const uint2* rect, int tiles_x, uint32_t tile_base, uint32_t* tile_ids,
                       uint32_t* gids, hipStream_t s);
void launch_tile_ranges(int64_t P, const uint32_t* tile_sorted, uint32_t n_tiles, uint32_t* ranges,
                        hipStream_t s);
void launch_fill_u32(uint32_t* p, uint32_t v, int64_t n, hipStream_t s);
void launch_fill_f32(float* p, float v, int64_t n, hipStream_t s);

// render.hip
// counters (optional, 5 x u64): see vcgs_count_read.
void launch_composite_fwd(const CamK& cam, const Splat* rec, const uint32_t* gids, const uint32_t* ranges,
                          const float* bg, float* color, float* depth, float* alpha, float* t_final,
                          uint32_t* n_contrib, unsigned long long* counters, hipStream_t s);
void launch_composite_bwd(const CamK& cam, const Splat* rec, const uint32_t* gids, const uint32_t* ranges,
                          const float* bg, const float* t_final, const uint32_t* n_contrib,
                          const float* dl_dc, const float* dl_dd, const float* dl_da, float* g2,
                          unsigned long long* counters, hipStream_t s);
// Process-wide kernel configuration (vcgs_set_option).
struct Options {
    int ppl_fwd = 1;  // pixels per lane of the forward compositing (1, 2, 4)
    int ppl_bwd = 1;  // pixels per lane of the backward compositing (1, 2, 4)
    int cull = 1;     // per-wave ellipse culling of tile-list entries
};
Options& options();
int l1_loss_blocks(int64_t npix);
// partial: l1_loss_blocks(npix) floats of scratch (only used when loss != nullptr)
void launch_l1_loss(int64_t npix, const float* c, const float* d, const float* tc, const float* td,
                    float w_depth, float* dl_dc, float* dl_dd, float* loss, float* partial, hipStream_t s);

// decode.hip
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
};
void launch_decode_fwd(const DecodeArgs& a, const vcgs_gaussian_buffers& out, hipStream_t s);
int decode_bwd_blocks(int64_t na);
__host__ __device__ int64_t decode_bwd_partial_floats(int k);
void launch_decode_bwd(const DecodeArgs& a, const vcgs_gaussian_buffers& dG, const vcgs_anchor_grads& out,
                       float* partial, int nblocks, hipStream_t s);

}  // namespace vcgs
