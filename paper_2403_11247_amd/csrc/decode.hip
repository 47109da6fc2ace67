// Anchor decode (paper Sec. 3.2, eqs. (7)-(9); mask eqs. (11)-(12); residual
// codebook eq. (14), first line) and its adjoint.
//
// The MLP input is the 32-d anchor feature, or with a camera centre x_c the
// 36-d [f_a, delta, d] of eq. (9) (delta = |x_a - x_c|, d = (x_a - x_c) / delta):
// the four view inputs are one more K step of the first layer's MFMA.
//
// The MLP h = ReLU(W1 f + b1), y = W2 h + b2 is the one dense contraction of
// the path and runs on FP32 MFMA (v_mfma_f32_16x16x4_f32): a wave decodes 16
// anchors at a time, anchors along the MFMA N dimension.  The second layer
// consumes the first layer's accumulators in place: its K index is ordered to
// match the accumulator layout (lane l holds rows 4*(l/16)+i of column l%16),
// so no data moves between the layers.  Outputs go through a wave-private LDS
// slab so the per-Gaussian activations are written coalesced, structure of
// arrays, Gaussian index = anchor * k + offset.
//
// Backward recomputes the forward MLP, forms dL/dy in LDS, and runs the three
// transposed products (dh = W2^T dy, df = W1^T dpre, and the weight gradients
// dW2 = dy h^T, dW1 = dpre f^T summed over anchors) on MFMA as well.  A block
// of four waves takes one 16-anchor group at a time and splits its steps over
// the waves (output tiles, feature tiles), so a group's chain of dependent
// steps is about a quarter as long as one wave's; every weight-gradient value
// has one owning lane, and the per-block partial rows are summed across blocks
// in a fixed order (deterministic).
#include "internal.h"

namespace vcgs {

typedef float v4f __attribute__((ext_vector_type(4)));

constexpr int kF = 32;
constexpr int kMaxK = 16;
constexpr int kMaxO = kMaxK * 11;
// Row stride of the per-wave [16 anchors][k * 11] output buffers for OT
// 16-row output tiles (padded by one float against bank conflicts).
constexpr int lds_o(int OT) { return OT * 16 + 1; }

__device__ __forceinline__ v4f mfma4(float a, float b, v4f c)
{
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ float sigm(float x) { return 1.0f / (1.0f + __expf(-x)); }

__device__ __forceinline__ void wsync()
{
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// Block barrier that orders LDS only: the waves' global stores (per-anchor
// outputs) stay in flight across it, since no wave reads another's global
// writes.  (__syncthreads would wait for every outstanding store first.)
__device__ __forceinline__ void lds_barrier()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Codebook row of Gaussian g at stage s; indices outside [0, size) are clamped.
__device__ __forceinline__ int code_index(const DecodeArgs& a, int s, int64_t n, int64_t g)
{
    const int i = a.idx[(int64_t)s * n + g];
    return i < 0 ? 0 : (i >= a.cb_size ? a.cb_size - 1 : i);
}

// Gaussian attributes of one (anchor, offset) from the MLP outputs y[0..10].
struct Decoded {
    float o_raw, c[3], s_raw[3], q[4], v[7];
    bool keep;
};

// mask_logit: the Gaussian's mask logit (read only when a.mask_logit is set).
__device__ __forceinline__ Decoded decode_one(const DecodeArgs& a, const float* y, int64_t g, float mask_logit)
{
    Decoded d;
    d.o_raw = sigm(y[0]);
#pragma unroll
    for (int i = 0; i < 3; ++i) d.c[i] = sigm(y[1 + i]);
    if (a.books) {
#pragma unroll
        for (int i = 0; i < 7; ++i) d.v[i] = 0.0f;
        const int64_t n = a.na * a.k;
        for (int s = 0; s < a.stages; ++s) {
            const float* row = a.books + ((int64_t)s * a.cb_size + code_index(a, s, n, g)) * 7;
#pragma unroll
            for (int i = 0; i < 7; ++i) d.v[i] += row[i];
        }
    } else {
#pragma unroll
        for (int i = 0; i < 7; ++i) d.v[i] = y[4 + i];
    }
#pragma unroll
    for (int i = 0; i < 3; ++i) d.s_raw[i] = __expf(d.v[i]);
#pragma unroll
    for (int i = 0; i < 4; ++i) d.q[i] = d.v[3 + i];
    d.keep = a.mask_logit ? (mask_logit > a.mask_thr) : true;
    return d;
}

// View input c of anchor an for the camera centre cam (eq. (9)): c = 0 the
// distance, 1..3 the unit direction.
__device__ __forceinline__ float view_input(const DecodeArgs& a, const float* cam, int64_t an, int c)
{
    const float vx = a.xa[an] - cam[0], vy = a.xa[a.na + an] - cam[1], vz = a.xa[2 * a.na + an] - cam[2];
    const float dist = sqrtf(vx * vx + vy * vy + vz * vz);
    return c == 0 ? dist : (c == 1 ? vx : (c == 2 ? vy : vz)) / dist;
}

// Block-shared copies of the MLP weights, read at their point of use rather
// than held in registers: W2 rows padded to kW2S floats (rows at or beyond O
// zero), W1 rows padded to kW1S floats (columns at or beyond in_dim zero).
constexpr int kW2S = 36;
constexpr int kW1S = 52;

// First layer for 16 anchors; returns the pre-activations in accumulator layout
// and, with the view input, this lane's view value (anchor lane % 16, input lane / 16).
__device__ __forceinline__ void layer1_lds(const float* w1s, const DecodeArgs& a, const float* cam, int64_t an,
                                           bool valid, int lane, v4f (&d1)[2], float& vin)
{
    d1[0] = v4f{0.f, 0.f, 0.f, 0.f};
    d1[1] = v4f{0.f, 0.f, 0.f, 0.f};
    const float* r0 = w1s + (lane & 15) * kW1S + (lane >> 4);
    const float* r1 = r0 + 16 * kW1S;
#pragma unroll
    for (int ks = 0; ks < 8; ++ks) {
        const float b = valid ? a.feat[an * kF + ks * 4 + (lane >> 4)] : 0.0f;
        d1[0] = mfma4(r0[ks * 4], b, d1[0]);
        d1[1] = mfma4(r1[ks * 4], b, d1[1]);
    }
    vin = 0.0f;
    if (a.in_dim > kF) {  // uniform
        vin = valid ? view_input(a, cam, an, lane >> 4) : 0.0f;
        d1[0] = mfma4(r0[32], vin, d1[0]);
        d1[1] = mfma4(r1[32], vin, d1[1]);
    }
}

// View v's block of a stacked per-view Gaussian set of n Gaussians per view.
__device__ __forceinline__ vcgs_gaussian_buffers view_block(const vcgs_gaussian_buffers& g, int v, int64_t n)
{
    vcgs_gaussian_buffers r;
    r.mean = g.mean ? g.mean + 3 * v * n : nullptr;
    r.scale = g.scale ? g.scale + 3 * v * n : nullptr;
    r.quat = g.quat ? g.quat + 4 * v * n : nullptr;
    r.opacity = g.opacity ? g.opacity + v * n : nullptr;
    r.color = g.color ? g.color + 3 * v * n : nullptr;
    return r;
}

// Per-anchor outputs of the backward: the first view stores, later views add.
__device__ __forceinline__ void put(float* p, bool first, float x) { *p = first ? x : *p + x; }

// Block-wide copy of the weights into LDS (ends with a block barrier).
template <int OT>
__device__ __forceinline__ void fill_weights(const DecodeArgs& a, float* w2s, float* w1s, float* b2s, float* b1s)
{
    const int O = a.k * 11;
    for (int i = threadIdx.x; i < OT * 16 * kW2S; i += blockDim.x) {
        const int m = i / kW2S, c = i - m * kW2S;
        w2s[i] = (m < O && c < kF) ? a.W2[m * kF + c] : 0.0f;
    }
    for (int i = threadIdx.x; i < kF * kW1S; i += blockDim.x) {
        const int r = i / kW1S, c = i - r * kW1S;
        w1s[i] = c < a.in_dim ? a.W1[r * a.in_dim + c] : 0.0f;
    }
    for (int i = threadIdx.x; i < OT * 16; i += blockDim.x) b2s[i] = i < O ? a.b2[i] : 0.0f;
    if (threadIdx.x < kF) b1s[threadIdx.x] = a.b1[threadIdx.x];
    __syncthreads();
}

// Second layer for 16 anchors from the LDS weights: y = W2 h + b2 into the
// wave's [16 anchors][O] buffer.
template <int OT, int LO>
__device__ __forceinline__ void layer2_lds(const float* w2s, const float* b2s, const float (&h)[2][4], int O, int lane,
                                           float (*yw)[LO])
{
#pragma unroll
    for (int t = 0; t < OT; ++t) {
        v4f d2 = {0.f, 0.f, 0.f, 0.f};
        const float* wr = w2s + (t * 16 + (lane & 15)) * kW2S + 4 * (lane >> 4);
#pragma unroll
        for (int st = 0; st < 8; ++st) d2 = mfma4(wr[(st >> 2) * 16 + (st & 3)], h[st >> 2][st & 3], d2);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int m = t * 16 + 4 * (lane >> 4) + i;
            if (m < O) yw[lane & 15][m] = d2[i] + b2s[m];
        }
    }
}

template <int OT>
__global__ void __launch_bounds__(256) k_decode_fwd(DecodeArgs a, float* __restrict__ mean0, float* __restrict__ scale0,
                                                    float* __restrict__ quat0, float* __restrict__ opac0,
                                                    float* __restrict__ color0)
{
    constexpr int LO = lds_o(OT);
    __shared__ float ys[4][16][LO];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int O = a.k * 11;
    __shared__ __align__(16) float w2s[OT * 16 * kW2S];
    __shared__ float w1s[kF * kW1S];
    __shared__ float b2s[OT * 16];
    __shared__ float b1s[kF];
    fill_weights<OT>(a, w2s, w1s, b2s, b1s);
    const int64_t n = a.na * a.k;
    const int64_t groups = (a.na + 15) / 16;
    // work items: (view, 16-anchor group), view-major
    for (int64_t it = (int64_t)blockIdx.x * 4 + wave; it < groups * a.views; it += (int64_t)gridDim.x * 4) {
        const int v = (int)(it / groups);
        const int64_t grp = it - v * groups;
        const int64_t a0 = grp * 16;
        const int64_t an = a0 + (lane & 15);
        float* mean = mean0 + 3 * v * n;
        float* scale = scale0 + 3 * v * n;
        float* quat = quat0 + 4 * v * n;
        float* opac = opac0 + v * n;
        float* color = color0 + 3 * v * n;
        v4f d1[2];
        float vin;
        layer1_lds(w1s, a, a.cam[v], an, an < a.na, lane, d1, vin);
        float h[2][4];
#pragma unroll
        for (int mt = 0; mt < 2; ++mt)
#pragma unroll
            for (int i = 0; i < 4; ++i) h[mt][i] = fmaxf(d1[mt][i] + b1s[mt * 16 + 4 * (lane >> 4) + i], 0.0f);
        wsync();
        layer2_lds<OT, LO>(w2s, b2s, h, O, lane, ys[wave]);
        wsync();
        for (int e = lane; e < 16 * a.k; e += 64) {
            const int al = e / a.k, off = e - al * a.k;
            const int64_t anc = a0 + al;
            if (anc >= a.na) continue;
            const int64_t g = anc * a.k + off;
            const Decoded d = decode_one(a, &ys[wave][al][off * 11], g, a.mask_logit ? a.mask_logit[g] : 0.0f);
            opac[g] = d.keep ? d.o_raw : 0.0f;
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                color[i * n + g] = d.c[i];
                scale[i * n + g] = d.keep ? d.s_raw[i] : 0.0f;
                const float* O3 = a.offset + g * 3;
                mean[i * n + g] = a.xa[i * a.na + anc] + O3[i] * a.scaling[i * a.na + anc];
            }
#pragma unroll
            for (int i = 0; i < 4; ++i) quat[i * n + g] = d.q[i];
        }
    }
}

static int out_tiles(int k) { return (k * 11 + 15) / 16; }

// Forward grid cap: three blocks per CU (LDS bound); each block copies the
// weights into LDS once, so waves that stride over several 16-anchor groups
// amortise that copy.
constexpr int kFwdMaxBlocks = 768;

void launch_decode_fwd(const DecodeArgs& a, const vcgs_gaussian_buffers& out, hipStream_t s)
{
    if (a.na <= 0) return;
    const int64_t items = (a.na + 15) / 16 * a.views;
    const int blocks = (int)std::min<int64_t>((items + 3) / 4, kFwdMaxBlocks);
#define VCGS_DEC_FWD(OT)                                                                                        \
    case OT:                                                                                                    \
        k_decode_fwd<OT><<<blocks, 256, 0, s>>>(a, out.mean, out.scale, out.quat, out.opacity, out.color);      \
        break;
    switch (out_tiles(a.k)) {
        VCGS_DEC_FWD(1) VCGS_DEC_FWD(2) VCGS_DEC_FWD(3) VCGS_DEC_FWD(4) VCGS_DEC_FWD(5) VCGS_DEC_FWD(6)
        VCGS_DEC_FWD(7) VCGS_DEC_FWD(8) VCGS_DEC_FWD(9) VCGS_DEC_FWD(10) VCGS_DEC_FWD(11)
        default: break;
    }
#undef VCGS_DEC_FWD
}

// ---------------------------------------------------------------------------
// Backward
// ---------------------------------------------------------------------------
constexpr int kBwdWaves = 4;

// Partial row of one block: dW2 [O][32], db2 [O], dW1 [32][in_dim], db1 [32], dL/dcam [views][3].
__host__ __device__ int64_t decode_bwd_partial_floats(int k, int in_dim, int views)
{
    return (int64_t)k * 11 * kF + k * 11 + (int64_t)kF * in_dim + kF + 3 * views;
}

// Output tiles (16 rows of the k * 11 MLP outputs) of wave w: t = w, w + 4, w + 8.
constexpr int wave_tiles(int OT) { return (OT + kBwdWaves - 1) / kBwdWaves; }

// LDS of one block of the backward, in floats: the weights, y / dL/dy of the
// group [16][lds_o], the per-entry staging [256][6], h, dL/dpre and view inputs
// [16][33], the four waves' partial dL/dh [4][8][64], the camera-centre sums.
constexpr int bwd_lds_floats(int OT)
{
    return OT * 16 * kW2S + kF * kW1S + OT * 16 + kF + 16 * lds_o(OT) + 256 * 6 + 2 * 16 * (kF + 1) + 16 * 4 +
           kBwdWaves * 8 * 64 + kDecodeMaxViews * 3;
}

int decode_bwd_blocks(int64_t na, int k)
{
    const int64_t groups = (na + 15) / 16;
    const int ot = std::min(std::max(out_tiles(k), 1), 11);
    const int per_cu = std::max(1, (160 * 1024) / (bwd_lds_floats(ot) * 4));  // blocks per CU that the LDS admits
    return (int)std::max<int64_t>(1, std::min<int64_t>(groups, (int64_t)256 * per_cu));
}

// One 16-anchor group at a time per block, its work spread over the four
// waves with block barriers between the steps:
//   1. every thread loads one (anchor, offset) entry's inputs and attribute
//      gradients (16 k <= 256 entries) and stages the mean gradient and its
//      offset product; wave 2 then sums them per anchor (anchor position and
//      scaling gradients);
//   2. every wave recomputes the first layer (16 MFMA steps; it needs h and
//      the pre-activations in its own registers) and the second layer for its
//      output tiles t = w, w + 4, ... into the group's y buffer;
//   3. every thread turns its entry's y into dL/dy in place (sigmoid and exp
//      adjoints, mask and codebook gradients);
//   4. each wave accumulates dW2 = dy h^T and db2 for its tiles and the part
//      of dh = W2^T dy that its tiles contribute;
//   5. every wave adds the four partial dh in wave order and applies the ReLU
//      mask; waves 0 and 1 form df = W1^T dpre for features 0-15 and 16-31 (the
//      anchor-feature gradients), wave 2 the view rows (camera-centre
//      gradient);
//   6. waves 0-2 accumulate dW1 = dpre f^T for their feature tile, wave 3 db1.
// Every weight-gradient element has one owning lane in the block, so the
// block's partial row is written without a block reduction, and the partial
// rows are summed over blocks in a fixed order by k_decode_bwd_reduce
// (deterministic).  With several camera centres the block takes its group
// through every view in turn: per-anchor outputs are stored by the first view
// and added by the later ones, always by the same lane.
template <int OT>
__global__ void __launch_bounds__(64 * kBwdWaves, 3) k_decode_bwd(DecodeArgs a, vcgs_gaussian_buffers dG,
                                                              vcgs_anchor_grads out, float* __restrict__ partial,
                                                              float* __restrict__ dvbuf)
{
    constexpr int LO = lds_o(OT);
    constexpr int WT = wave_tiles(OT);
    __shared__ __align__(16) float w2s[OT * 16 * kW2S];
    __shared__ float w1s[kF * kW1S];
    __shared__ float b2s[OT * 16];
    __shared__ float b1s[kF];
    __shared__ float ys[16][LO];          // y, then dL/dy in place
    __shared__ float stg[256 * 6];        // per entry: dL/dmean, dL/dmean * offset
    __shared__ float hs[16][kF + 1];      // h [anchor][hidden]
    __shared__ float ps[16][kF + 1];      // dL/dpre [anchor][hidden]
    __shared__ float vs[16][4];           // view inputs [anchor][distance, direction]
    __shared__ float dhp[kBwdWaves][8][64];  // partial dL/dh per wave, accumulator layout
    __shared__ float camw[kDecodeMaxViews * 3];  // dL/d camera centre per view (wave 2)
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int O = a.k * 11;
    const int64_t n = a.na * a.k;
    const bool view = a.in_dim > kF;  // uniform
    fill_weights<OT>(a, w2s, w1s, b2s, b1s);
    if (threadIdx.x < kDecodeMaxViews * 3) camw[threadIdx.x] = 0.0f;
    v4f accW2[WT][2], accW1[2];
#pragma unroll
    for (int j = 0; j < WT; ++j) accW2[j][0] = accW2[j][1] = v4f{0.f, 0.f, 0.f, 0.f};
    accW1[0] = accW1[1] = v4f{0.f, 0.f, 0.f, 0.f};
    float accB2 = 0.0f, accB1 = 0.0f;
    const int e = threadIdx.x;  // this thread's (anchor, offset) entry of the group
    const int eal = e / a.k, eoff = e - eal * a.k;
    const int ft = wave;        // df / dW1 feature tile of waves 0-2

    const int64_t groups = (a.na + 15) / 16;
    for (int64_t grp = blockIdx.x; grp < groups; grp += gridDim.x) {
        const int64_t a0 = grp * 16;
        const int64_t an = a0 + (lane & 15);  // the anchor of this lane's MFMA column
        const bool avalid = an < a.na;
        const int64_t eanc = a0 + eal;
        const bool eok = e < 16 * a.k && eanc < a.na;
        const int64_t g = eanc * a.k + eoff;
        // anchor features: the first layer's B operand (8 per lane) and, for
        // waves 0-1, the dW1 B operand of their feature tile (4 per lane)
        float fb[8], fw[4];
#pragma unroll
        for (int ks = 0; ks < 8; ++ks) fb[ks] = avalid ? a.feat[an * kF + ks * 4 + (lane >> 4)] : 0.0f;
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) {
            const int64_t anc = a0 + ks * 4 + (lane >> 4);
            fw[ks] = (ft < 2 && anc < a.na) ? a.feat[anc * kF + ft * 16 + (lane & 15)] : 0.0f;
        }
        const float sc0 = (eok && out.offset) ? a.scaling[eanc] : 0.0f;
        const float sc1 = (eok && out.offset) ? a.scaling[a.na + eanc] : 0.0f;
        const float sc2 = (eok && out.offset) ? a.scaling[2 * a.na + eanc] : 0.0f;
        const float of0 = eok ? a.offset[g * 3] : 0.0f;
        const float of1 = eok ? a.offset[g * 3 + 1] : 0.0f;
        const float of2 = eok ? a.offset[g * 3 + 2] : 0.0f;
        const float mlog = (eok && a.mask_logit) ? a.mask_logit[g] : 0.0f;
        for (int v = 0; v < a.views; ++v) {
            const bool first = v == 0;
            const vcgs_gaussian_buffers dGv = view_block(dG, v, n);
            lds_barrier();  // the previous group's or view's LDS is no longer read
            // ---- 1. this entry's gradients; per-anchor sums
            float dm[3], pg[11];
            dm[0] = (eok && dGv.mean) ? dGv.mean[g] : 0.0f;
            dm[1] = (eok && dGv.mean) ? dGv.mean[n + g] : 0.0f;
            dm[2] = (eok && dGv.mean) ? dGv.mean[2 * n + g] : 0.0f;
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                pg[i] = (eok && dGv.scale) ? dGv.scale[i * n + g] : 0.0f;
                pg[3 + i] = (eok && dGv.color) ? dGv.color[i * n + g] : 0.0f;
            }
#pragma unroll
            for (int i = 0; i < 4; ++i) pg[6 + i] = (eok && dGv.quat) ? dGv.quat[i * n + g] : 0.0f;
            pg[10] = (eok && dGv.opacity) ? dGv.opacity[g] : 0.0f;
            if (e < 16 * a.k) {
                stg[e * 6 + 0] = dm[0];
                stg[e * 6 + 1] = dm[1];
                stg[e * 6 + 2] = dm[2];
                stg[e * 6 + 3] = dm[0] * of0;
                stg[e * 6 + 4] = dm[1] * of1;
                stg[e * 6 + 5] = dm[2] * of2;
            }
            if (eok && out.offset) {
                put(out.offset + g * 3, first, dm[0] * sc0);
                put(out.offset + g * 3 + 1, first, dm[1] * sc1);
                put(out.offset + g * 3 + 2, first, dm[2] * sc2);
            }
            // ---- 2. first layer (every wave), second layer for this wave's tiles
            v4f d1[2] = {v4f{0.f, 0.f, 0.f, 0.f}, v4f{0.f, 0.f, 0.f, 0.f}};
            {
                const float* r0 = w1s + (lane & 15) * kW1S + (lane >> 4);
                const float* r1 = r0 + 16 * kW1S;
#pragma unroll
                for (int ks = 0; ks < 8; ++ks) {
                    d1[0] = mfma4(r0[ks * 4], fb[ks], d1[0]);
                    d1[1] = mfma4(r1[ks * 4], fb[ks], d1[1]);
                }
                if (view) {
                    const float vin = avalid ? view_input(a, a.cam[v], an, lane >> 4) : 0.0f;
                    d1[0] = mfma4(r0[32], vin, d1[0]);
                    d1[1] = mfma4(r1[32], vin, d1[1]);
                    if (wave == 2) vs[lane & 15][lane >> 4] = vin;
                }
            }
            float pre[2][4], h[2][4];
#pragma unroll
            for (int mt = 0; mt < 2; ++mt)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    pre[mt][i] = d1[mt][i] + b1s[mt * 16 + 4 * (lane >> 4) + i];
                    h[mt][i] = avalid ? fmaxf(pre[mt][i], 0.0f) : 0.0f;
                }
            if (wave == 0) {
#pragma unroll
                for (int mt = 0; mt < 2; ++mt)
#pragma unroll
                    for (int i = 0; i < 4; ++i) hs[lane & 15][mt * 16 + 4 * (lane >> 4) + i] = h[mt][i];
            }
#pragma unroll
            for (int j = 0; j < WT; ++j) {
                const int t = wave + kBwdWaves * j;
                if (t < OT) {
                    v4f d2 = {0.f, 0.f, 0.f, 0.f};
                    const float* wr = w2s + (t * 16 + (lane & 15)) * kW2S + 4 * (lane >> 4);
#pragma unroll
                    for (int st = 0; st < 8; ++st) d2 = mfma4(wr[(st >> 2) * 16 + (st & 3)], h[st >> 2][st & 3], d2);
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const int m = t * 16 + 4 * (lane >> 4) + i;
                        if (m < O) ys[lane & 15][m] = d2[i] + b2s[m];
                    }
                }
            }
            lds_barrier();
            if (wave == 2 && lane < 16 && a0 + lane < a.na) {
                // anchor position and scaling gradients: sums over the offsets in order
                const int64_t anc = a0 + lane;
                float dx[3] = {0.0f, 0.0f, 0.0f}, dls[3] = {0.0f, 0.0f, 0.0f};
                for (int off = 0; off < a.k; ++off) {
                    const float* q = stg + (lane * a.k + off) * 6;
#pragma unroll
                    for (int i = 0; i < 3; ++i) {
                        dx[i] += q[i];
                        dls[i] += q[3 + i];
                    }
                }
#pragma unroll
                for (int i = 0; i < 3; ++i) {
                    if (out.scaling) put(out.scaling + i * a.na + anc, first, dls[i]);
                    if (out.xa) put(out.xa + i * a.na + anc, first, dx[i]);
                }
            }
            // ---- 3. dL/dy of this entry, in place
            if (e < 16 * a.k) {
                float* dy = &ys[eal][eoff * 11];
                if (!eok) {
#pragma unroll
                    for (int i = 0; i < 11; ++i) dy[i] = 0.0f;
                } else {
                    const Decoded d = decode_one(a, dy, g, mlog);
                    float ds[3] = {pg[0], pg[1], pg[2]};
                    float dop = pg[10];
                    if (a.mask_logit) {
                        float gm = 0.0f;
                        if (d.keep) {
                            const float sg = sigm(mlog);
                            gm = sg * (1.0f - sg) * (ds[0] * d.s_raw[0] + ds[1] * d.s_raw[1] + ds[2] * d.s_raw[2] + dop * d.o_raw);
                        } else {
                            ds[0] = ds[1] = ds[2] = 0.0f;
                            dop = 0.0f;
                        }
                        if (out.mask_logit) put(out.mask_logit + g, first, gm);
                    }
                    dy[0] = dop * d.o_raw * (1.0f - d.o_raw);
#pragma unroll
                    for (int i = 0; i < 3; ++i) dy[1 + i] = pg[3 + i] * d.c[i] * (1.0f - d.c[i]);
                    float dv[7];
#pragma unroll
                    for (int i = 0; i < 3; ++i) dv[i] = ds[i] * d.s_raw[i];
#pragma unroll
                    for (int i = 0; i < 4; ++i) dv[3 + i] = pg[6 + i];
                    if (a.books) {
#pragma unroll
                        for (int i = 0; i < 7; ++i) dy[4 + i] = 0.0f;
                        if (out.books && dvbuf) {  // per-Gaussian rows, summed per code by k_books_partial
#pragma unroll
                            for (int i = 0; i < 7; ++i) put(dvbuf + g * 8 + i, first, dv[i]);
                        } else if (out.books) {
                            for (int s = 0; s < a.stages; ++s) {
                                float* row = out.books + ((int64_t)s * a.cb_size + code_index(a, s, n, g)) * 7;
#pragma unroll
                                for (int i = 0; i < 7; ++i) atomicAdd(row + i, dv[i]);
                            }
                        }
                    } else {
#pragma unroll
                        for (int i = 0; i < 7; ++i) dy[4 + i] = dv[i];
                    }
                }
            }
            // entries of anchors beyond the group's 16 * k slots are never read
            lds_barrier();
            // ---- 4. db2, dW2 = dy h^T and this wave's share of dh = W2^T dy
            if (e < O) {
                float sacc = 0.0f;
#pragma unroll
                for (int al = 0; al < 16; ++al) sacc += ys[al][e];
                accB2 += sacc;
            }
            v4f dh[2] = {v4f{0.f, 0.f, 0.f, 0.f}, v4f{0.f, 0.f, 0.f, 0.f}};
#pragma unroll
            for (int j = 0; j < WT; ++j) {
                const int t = wave + kBwdWaves * j;
                if (t < OT) {
#pragma unroll
                    for (int ks = 0; ks < 4; ++ks) {
                        const int al = ks * 4 + (lane >> 4);
                        const int m = t * 16 + (lane & 15);
                        const float av = m < O ? ys[al][m] : 0.0f;
                        accW2[j][0] = mfma4(av, hs[al][lane & 15], accW2[j][0]);
                        accW2[j][1] = mfma4(av, hs[al][16 + (lane & 15)], accW2[j][1]);
                    }
#pragma unroll
                    for (int kq = 0; kq < 4; ++kq) {
                        const int ks = t * 4 + kq;
                        const int m = ks * 4 + (lane >> 4);
                        const float bv = m < O ? ys[lane & 15][m] : 0.0f;
                        const float* wr = w2s + m * kW2S + (lane & 15);
                        dh[0] = mfma4(wr[0], bv, dh[0]);
                        dh[1] = mfma4(wr[16], bv, dh[1]);
                    }
                }
            }
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                dhp[wave][i][lane] = dh[0][i];
                dhp[wave][4 + i][lane] = dh[1][i];
            }
            lds_barrier();
            // ---- 5. dpre (the four partial dh in wave order), df
            float dpre[2][4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const float s0 = ((dhp[0][i][lane] + dhp[1][i][lane]) + dhp[2][i][lane]) + dhp[3][i][lane];
                const float s1 = ((dhp[0][4 + i][lane] + dhp[1][4 + i][lane]) + dhp[2][4 + i][lane]) + dhp[3][4 + i][lane];
                dpre[0][i] = (avalid && pre[0][i] > 0.0f) ? s0 : 0.0f;
                dpre[1][i] = (avalid && pre[1][i] > 0.0f) ? s1 : 0.0f;
            }
            if (wave == 3) {
#pragma unroll
                for (int mt = 0; mt < 2; ++mt)
#pragma unroll
                    for (int i = 0; i < 4; ++i) ps[lane & 15][mt * 16 + 4 * (lane >> 4) + i] = dpre[mt][i];
            }
            if (ft < 2 || (ft == 2 && view)) {
                v4f df = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int st = 0; st < 8; ++st) {
                    const float* wr = w1s + ((st >> 2) * 16 + 4 * (lane >> 4) + (st & 3)) * kW1S + ft * 16 + (lane & 15);
                    df = mfma4(wr[0], dpre[st >> 2][st & 3], df);
                }
                if (ft < 2) {
                    if (out.feat && avalid) {
#pragma unroll
                        for (int i = 0; i < 4; ++i) put(out.feat + an * kF + ft * 16 + 4 * (lane >> 4) + i, first, df[i]);
                    }
                } else {
                    float dc[3] = {0.0f, 0.0f, 0.0f};  // this anchor's share of dL/d camera centre
                    if (lane < 16 && avalid) {
                        // lanes 0-15 hold rows 32..35 (dL/d distance, dL/d direction) of anchor `lane`:
                        // dL/dv = dL/ddelta d + (dL/dd - (dL/dd . d) d) / delta,  v = x_a - x_c
                        const float dist = vs[lane][0];
                        const float d0 = vs[lane][1], d1v = vs[lane][2], d2 = vs[lane][3];
                        const float gd = df[1] * d0 + df[2] * d1v + df[3] * d2;
                        const float dv[3] = {df[0] * d0 + (df[1] - gd * d0) / dist,
                                             df[0] * d1v + (df[2] - gd * d1v) / dist,
                                             df[0] * d2 + (df[3] - gd * d2) / dist};
#pragma unroll
                        for (int i = 0; i < 3; ++i) {
                            if (out.xa) out.xa[i * a.na + an] += dv[i];
                            dc[i] = -dv[i];
                        }
                    }
                    // the 16 anchors' sum (lanes 0-15), added to view v's total
#pragma unroll
                    for (int i = 0; i < 3; ++i)
#pragma unroll
                        for (int o = 8; o > 0; o >>= 1) dc[i] += __shfl_xor(dc[i], o, 16);
                    if (lane == 0) {
#pragma unroll
                        for (int i = 0; i < 3; ++i) camw[v * 3 + i] += dc[i];
                    }
                }
            }
            lds_barrier();
            // ---- 6. dW1 += dpre f^T (waves 0-2, their feature tile), db1 (wave 3)
            if (ft < 2 || (ft == 2 && view)) {
#pragma unroll
                for (int ks = 0; ks < 4; ++ks) {
                    const int al = ks * 4 + (lane >> 4);
                    const float f = ft < 2 ? fw[ks] : ((lane & 15) < 4 ? vs[al][lane & 15] : 0.0f);
                    accW1[0] = mfma4(ps[al][lane & 15], f, accW1[0]);
                    accW1[1] = mfma4(ps[al][16 + (lane & 15)], f, accW1[1]);
                }
            } else if (wave == 3 && lane < kF) {
                float sacc = 0.0f;
#pragma unroll
                for (int al = 0; al < 16; ++al) sacc += ps[al][lane];
                accB1 += sacc;
            }
        }
    }
    lds_barrier();
    // partial row: dW2 [O][32] | db2 [O] | dW1 [32][in_dim] | db1 [32] | dcam [views][3]
    const int64_t PF = decode_bwd_partial_floats(a.k, a.in_dim, a.views);
    const int oB2 = O * kF, oW1 = oB2 + O, oB1 = oW1 + kF * a.in_dim, oCam = oB1 + kF;
    float* row = partial + (int64_t)blockIdx.x * PF;
#pragma unroll
    for (int j = 0; j < WT; ++j) {
        const int t = wave + kBwdWaves * j;
        if (t < OT) {
#pragma unroll
            for (int nt = 0; nt < 2; ++nt)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int m = t * 16 + 4 * (lane >> 4) + i;
                    if (m < O) row[m * kF + nt * 16 + (lane & 15)] = accW2[j][nt][i];
                }
        }
    }
    if (e < O) row[oB2 + e] = accB2;
    if (ft < 2 || (ft == 2 && view)) {
        const int col = ft * 16 + (lane & 15);
        if (col < a.in_dim) {
#pragma unroll
            for (int nt = 0; nt < 2; ++nt)
#pragma unroll
                for (int i = 0; i < 4; ++i) row[oW1 + (nt * 16 + 4 * (lane >> 4) + i) * a.in_dim + col] = accW1[nt][i];
        }
    } else if (wave == 3 && lane < kF) {
        row[oB1 + lane] = accB1;
    }
    if (threadIdx.x < 3 * a.views) row[oCam + threadIdx.x] = camw[threadIdx.x];
}

// Sum of the per-block partial rows: each block owns 64 consecutive outputs;
// its 16 waves add interleaved sixteenths of the rows and combine in wave order.
constexpr int kRedWaves = 16;
__global__ void __launch_bounds__(64 * kRedWaves) k_decode_bwd_reduce(const float* __restrict__ partial, int nblocks, int64_t PF,
                                                           int O, int in_dim, float* __restrict__ dW2,
                                                           float* __restrict__ db2, float* __restrict__ dW1,
                                                           float* __restrict__ db1, float* __restrict__ dcam)
{
    __shared__ float acc[kRedWaves][64];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t i = (int64_t)blockIdx.x * 64 + lane;
    float s = 0.0f;
    if (i < PF) {
#pragma unroll 4
        for (int b = wave; b < nblocks; b += kRedWaves) s += partial[(int64_t)b * PF + i];
    }
    acc[wave][lane] = s;
    __syncthreads();
    if (wave != 0 || i >= PF) return;
    s = acc[0][lane];
#pragma unroll
    for (int w = 1; w < kRedWaves; ++w) s += acc[w][lane];
    const int64_t oW2 = (int64_t)O * kF, oB2 = oW2 + O, oW1 = oB2 + (int64_t)kF * in_dim, oB1 = oW1 + kF;
    if (i < oW2) { if (dW2) dW2[i] = s; }
    else if (i < oB2) { if (db2) db2[i - oW2] = s; }
    else if (i < oW1) { if (dW1) dW1[i - oB2] = s; }
    else if (i < oB1) { if (db1) db1[i - oW1] = s; }
    else { if (dcam && in_dim > kF) dcam[i - oB1] = s; }
}

// ---------------------------------------------------------------------------
// Pose share of the camera-centre input (eq. (9)): the centre x_c = -R^T t of
// a world-to-camera pose moves by -R^T rho under the left perturbation
// exp(xi^) {R|t}, so dL/drho gains -R dL/dx_c and dL/dphi nothing.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(64) k_centre_pose_grad(CentreTab t, const float* __restrict__ dcam,
                                                         float* __restrict__ dpose)
{
    const int v = threadIdx.x / 3, i = threadIdx.x % 3;
    if (v >= t.views) return;
    const float* R = t.R[v];
    const float* g = dcam + 3 * v;
    dpose[6 * v + i] -= R[3 * i] * g[0] + R[3 * i + 1] * g[1] + R[3 * i + 2] * g[2];
}

void launch_centre_pose_grad(const CentreTab& t, const float* dcam, float* dpose, hipStream_t s)
{
    if (t.views > 0) k_centre_pose_grad<<<1, 64, 0, s>>>(t, dcam, dpose);
}

// ---------------------------------------------------------------------------
// Codebook gradient (straight-through sums of eq. (14)'s gathered rows)
// ---------------------------------------------------------------------------
// Each of 8192 rows of a 2 x 4096 codebook is shared by ~100 Gaussians of the
// room, so adding every Gaussian's 7 values to its rows with device atomics
// contends (0.32 ms of the room's decode backward).  Instead the backward
// stores each Gaussian's 7 values; every block then adds its share of the
// Gaussians into a stage's whole table in LDS (low contention: the rows are
// spread) and writes that table as its partial, and the partials are summed
// in block order.
constexpr int kBookThreads = 1024;
constexpr int kBookMaxBlocks = 256;

int books_grad_blocks(int64_t n)
{
    return (int)std::max<int64_t>(1, std::min<int64_t>((n + 4095) / 4096, kBookMaxBlocks));
}

__global__ void __launch_bounds__(kBookThreads) k_books_partial(DecodeArgs a, const float* __restrict__ dv,
                                                                float* __restrict__ partial)
{
    extern __shared__ float tab[];  // cb_size * 7
    const int64_t n = a.na * a.k;
    const int rows7 = a.cb_size * 7;
    for (int s = 0; s < a.stages; ++s) {
        for (int i = threadIdx.x; i < rows7; i += blockDim.x) tab[i] = 0.0f;
        __syncthreads();
        for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < n; g += (int64_t)gridDim.x * blockDim.x) {
            float* row = tab + code_index(a, s, n, g) * 7;
            const float4 v0 = *reinterpret_cast<const float4*>(dv + g * 8);
            const float4 v1 = *reinterpret_cast<const float4*>(dv + g * 8 + 4);
            atomicAdd(row + 0, v0.x); atomicAdd(row + 1, v0.y); atomicAdd(row + 2, v0.z); atomicAdd(row + 3, v0.w);
            atomicAdd(row + 4, v1.x); atomicAdd(row + 5, v1.y); atomicAdd(row + 6, v1.z);
        }
        __syncthreads();
        float* out = partial + ((int64_t)blockIdx.x * a.stages + s) * rows7;
        for (int i = threadIdx.x; i < rows7; i += blockDim.x) out[i] = tab[i];
        __syncthreads();
    }
}

__global__ void __launch_bounds__(256) k_books_reduce(const float* __restrict__ partial, int nblocks, int64_t per,
                                                      float* __restrict__ books_grad)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= per) return;
    float sacc = 0.0f;
    for (int b = 0; b < nblocks; ++b) sacc += partial[(int64_t)b * per + i];
    books_grad[i] = sacc;
}

// LDS bytes of k_books_partial's table; 0 when a codebook stage does not fit
// (the backward then adds to the rows with device atomics).
size_t books_lds_bytes(int cb_size)
{
    static int state[64] = {};  // per device: 0 unknown, 1 allowed, -1 refused
    const size_t bytes = (size_t)cb_size * 7 * sizeof(float);
    if (bytes > kBookLdsMax) return 0;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 0;
    if (state[dev] == 0)
        state[dev] = hipFuncSetAttribute((const void*)k_books_partial, hipFuncAttributeMaxDynamicSharedMemorySize,
                                         (int)kBookLdsMax) == hipSuccess ? 1 : -1;
    return state[dev] > 0 ? bytes : 0;
}

void launch_decode_bwd(const DecodeArgs& a, const vcgs_gaussian_buffers& dG, const vcgs_anchor_grads& out,
                       float* partial, int nblocks, float* dvbuf, float* book_partial, hipStream_t s)
{
    if (a.na <= 0) return;
    const bool books = out.books && a.books;
    const size_t lds = books && dvbuf && book_partial ? books_lds_bytes(a.cb_size) : 0;
    if (!lds) dvbuf = nullptr;
    if (books && !lds) launch_fill_f32(out.books, 0.0f, (int64_t)a.stages * a.cb_size * 7, s);
#define VCGS_DEC_BWD(OT)                                                                           \
    case OT:                                                                                       \
        k_decode_bwd<OT><<<nblocks, 64 * kBwdWaves, 0, s>>>(a, dG, out, partial, dvbuf);           \
        break;
    switch (out_tiles(a.k)) {
        VCGS_DEC_BWD(1) VCGS_DEC_BWD(2) VCGS_DEC_BWD(3) VCGS_DEC_BWD(4) VCGS_DEC_BWD(5) VCGS_DEC_BWD(6)
        VCGS_DEC_BWD(7) VCGS_DEC_BWD(8) VCGS_DEC_BWD(9) VCGS_DEC_BWD(10) VCGS_DEC_BWD(11)
        default: break;
    }
#undef VCGS_DEC_BWD
    const int64_t PF = decode_bwd_partial_floats(a.k, a.in_dim, a.views);
    k_decode_bwd_reduce<<<(unsigned)((PF + 63) / 64), 64 * kRedWaves, 0, s>>>(partial, nblocks, PF, a.k * 11, a.in_dim, out.W2,
                                                                   out.b2, out.W1, out.b1, out.cam);
    if (lds) {
        const int nbk = books_grad_blocks(a.na * a.k);
        const int64_t per = (int64_t)a.stages * a.cb_size * 7;
        k_books_partial<<<nbk, kBookThreads, lds, s>>>(a, dvbuf, book_partial);
        k_books_reduce<<<(unsigned)((per + 255) / 256), 256, 0, s>>>(book_partial, nbk, per, out.books);
    }
}

}  // namespace vcgs
