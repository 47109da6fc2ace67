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
// dW2 = dy h^T, dW1 = dpre f^T summed over anchors) on MFMA as well.  Weight
// gradients are summed per wave in registers, per block in a fixed wave order,
// and across blocks in a fixed order (deterministic).  The backward reads the
// weights from a block-shared LDS copy instead of registers, which leaves room
// for two waves per SIMD.
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

__device__ __forceinline__ Decoded decode_one(const DecodeArgs& a, const float* y, int64_t g)
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
    d.keep = a.mask_logit ? (a.mask_logit[g] > a.mask_thr) : true;
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
            const Decoded d = decode_one(a, &ys[wave][al][off * 11], g);
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
// Grid cap: two blocks per CU where registers and LDS allow two waves per SIMD
// (up to 8 output tiles), else one.
constexpr int kBwdMaxBlocks = 512;

// Partial row of one block: dW2 [O][32], db2 [O], dW1 [32][in_dim], db1 [32], dL/dcam [views][3].
__host__ __device__ int64_t decode_bwd_partial_floats(int k, int in_dim, int views)
{
    return (int64_t)k * 11 * kF + k * 11 + (int64_t)kF * in_dim + kF + 3 * views;
}

// Block reduction buffer, padded so that every lane owns a slot for each of
// its accumulators (no bounds tests, hence no per-slot branches): dW2 [OT*16][32],
// db2 [192], dW1 [32][48], db1 [64], dL/dcam [64].  The per-wave y buffers of
// a block double as it.
constexpr int kRedB2 = 192, kRedW1Cols = 48;
constexpr int red_b2(int OT) { return OT * 16 * kF; }
constexpr int red_w1(int OT) { return red_b2(OT) + kRedB2; }
constexpr int red_b1(int OT) { return red_w1(OT) + kF * kRedW1Cols; }
constexpr int red_cam(int OT) { return red_b1(OT) + 64; }
constexpr int bwd_red_floats(int OT) { return red_cam(OT) + 64; }
constexpr int bwd_smem_floats(int OT)
{
    return kBwdWaves * 16 * lds_o(OT) > bwd_red_floats(OT) ? kBwdWaves * 16 * lds_o(OT) : bwd_red_floats(OT);
}

int decode_bwd_blocks(int64_t na, int k)
{
    const int64_t groups = (na + 15) / 16;
    const int cap = out_tiles(k) <= 8 ? kBwdMaxBlocks : kBwdMaxBlocks / 2;
    return (int)std::max<int64_t>(1, std::min<int64_t>((groups + kBwdWaves - 1) / kBwdWaves, cap));
}

template <int OT>
__global__ void __launch_bounds__(64 * kBwdWaves, 2) k_decode_bwd(DecodeArgs a, vcgs_gaussian_buffers dG,
                                                               vcgs_anchor_grads out, float* __restrict__ partial,
                                                               float* __restrict__ dvbuf)
{
    // Each wave's [16 anchors][k * 11] outputs y are overwritten in place by
    // dL/dy (every slot is read before it is written, by the same lane); the
    // buffer also holds the block reduction at the end.
    constexpr int LO = lds_o(OT);
    __shared__ float smem[bwd_smem_floats(OT)];
    float (*ys)[16][LO] = reinterpret_cast<float (*)[16][LO]>(smem);
    float (*dys)[16][LO] = ys;
    __shared__ float hs[kBwdWaves][16][kF + 1];
    __shared__ float ps[kBwdWaves][16][kF + 1];
    __shared__ float vs[kBwdWaves][16][4];  // view inputs of the wave's 16 anchors
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int O = a.k * 11;
    const int64_t n = a.na * a.k;
    const bool view = a.in_dim > kF;  // uniform
    __shared__ __align__(16) float w2s[OT * 16 * kW2S];
    __shared__ float w1s[kF * kW1S];
    __shared__ float b2s[OT * 16];
    __shared__ float b1s[kF];
    fill_weights<OT>(a, w2s, w1s, b2s, b1s);
    v4f accW2[OT][2], accW1[2][3];
#pragma unroll
    for (int t = 0; t < OT; ++t) accW2[t][0] = accW2[t][1] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int nt = 0; nt < 2; ++nt)
#pragma unroll
        for (int ft = 0; ft < 3; ++ft) accW1[nt][ft] = v4f{0.f, 0.f, 0.f, 0.f};
    float accB2[(kMaxO + 63) / 64] = {0.f, 0.f, 0.f};
    float accB1 = 0.0f;
    __shared__ float camw[kBwdWaves][kDecodeMaxViews * 3];  // dL/d camera centre per wave and view
    if (lane < kDecodeMaxViews * 3) camw[wave][lane] = 0.0f;

    // each wave takes a 16-anchor group through every view in turn, so the
    // per-anchor outputs add up over the views without races
    const int64_t groups = (a.na + 15) / 16;
    for (int64_t grp = (int64_t)blockIdx.x * kBwdWaves + wave; grp < groups; grp += (int64_t)gridDim.x * kBwdWaves) {
        for (int v = 0; v < a.views; ++v) {
            const bool first = v == 0;
            const vcgs_gaussian_buffers dGv = view_block(dG, v, n);
            const int64_t a0 = grp * 16;
            const int64_t an = a0 + (lane & 15);
            const bool avalid = an < a.na;
            {
                // per-anchor sums over offsets (anchor position, scaling) and the offsets'
                // gradients: the (anchor, offset) pairs spread over the 64 lanes, their
                // contributions staged in the wave's y buffer (free until layer 2), then
                // added per anchor in offset order by 16 lanes
                float* stg = &ys[wave][0][0];  // 16 * LO >= 16 * k * 6 floats
                for (int e = lane; e < 16 * a.k; e += 64) {
                    const int al = e / a.k, off = e - al * a.k;
                    const int64_t anc = a0 + al;
                    float dm[3] = {0.0f, 0.0f, 0.0f}, dl[3] = {0.0f, 0.0f, 0.0f};
                    if (anc < a.na) {
                        const int64_t g = anc * a.k + off;
#pragma unroll
                        for (int i = 0; i < 3; ++i) {
                            dm[i] = dGv.mean ? dGv.mean[i * n + g] : 0.0f;
                            dl[i] = dm[i] * a.offset[g * 3 + i];
                        }
                        if (out.offset) {
#pragma unroll
                            for (int i = 0; i < 3; ++i) put(out.offset + g * 3 + i, first, dm[i] * a.scaling[i * a.na + anc]);
                        }
                    }
#pragma unroll
                    for (int i = 0; i < 3; ++i) {
                        stg[e * 6 + i] = dm[i];
                        stg[e * 6 + 3 + i] = dl[i];
                    }
                }
                wsync();
                if (lane < 16 && a0 + lane < a.na) {
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
                wsync();
            }
            v4f d1[2];
            float vin;
            layer1_lds(w1s, a, a.cam[v], an, avalid, lane, d1, vin);
            if (view) vs[wave][lane & 15][lane >> 4] = vin;
            float pre[2][4], h[2][4];
#pragma unroll
            for (int mt = 0; mt < 2; ++mt)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    pre[mt][i] = d1[mt][i] + b1s[mt * 16 + 4 * (lane >> 4) + i];
                    h[mt][i] = avalid ? fmaxf(pre[mt][i], 0.0f) : 0.0f;
                }
            wsync();
#pragma unroll
            for (int mt = 0; mt < 2; ++mt)
#pragma unroll
                for (int i = 0; i < 4; ++i) hs[wave][lane & 15][mt * 16 + 4 * (lane >> 4) + i] = h[mt][i];
            layer2_lds<OT, LO>(w2s, b2s, h, O, lane, ys[wave]);
            wsync();
            // dL/dy per (anchor, offset); codebook and mask gradients
            for (int e = lane; e < 16 * a.k; e += 64) {
                const int al = e / a.k, off = e - al * a.k;
                const int64_t anc = a0 + al;
                float* dy = &dys[wave][al][off * 11];
                if (anc >= a.na) {
#pragma unroll
                    for (int i = 0; i < 11; ++i) dy[i] = 0.0f;
                    continue;
                }
                const int64_t g = anc * a.k + off;
                const Decoded d = decode_one(a, &ys[wave][al][off * 11], g);
                float ds[3], dq[4], dc[3], dop;
#pragma unroll
                for (int i = 0; i < 3; ++i) {
                    ds[i] = dGv.scale ? dGv.scale[i * n + g] : 0.0f;
                    dc[i] = dGv.color ? dGv.color[i * n + g] : 0.0f;
                }
#pragma unroll
                for (int i = 0; i < 4; ++i) dq[i] = dGv.quat ? dGv.quat[i * n + g] : 0.0f;
                dop = dGv.opacity ? dGv.opacity[g] : 0.0f;
                if (a.mask_logit) {
                    const float m = a.mask_logit[g];
                    float gm = 0.0f;
                    if (d.keep) {
                        const float sg = sigm(m);
                        gm = sg * (1.0f - sg) * (ds[0] * d.s_raw[0] + ds[1] * d.s_raw[1] + ds[2] * d.s_raw[2] + dop * d.o_raw);
                    } else {
                        ds[0] = ds[1] = ds[2] = 0.0f;
                        dop = 0.0f;
                    }
                    if (out.mask_logit) put(out.mask_logit + g, first, gm);
                }
                dy[0] = dop * d.o_raw * (1.0f - d.o_raw);
#pragma unroll
                for (int i = 0; i < 3; ++i) dy[1 + i] = dc[i] * d.c[i] * (1.0f - d.c[i]);
                float dv[7];
#pragma unroll
                for (int i = 0; i < 3; ++i) dv[i] = ds[i] * d.s_raw[i];
#pragma unroll
                for (int i = 0; i < 4; ++i) dv[3 + i] = dq[i];
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
            wsync();
            // db2 and dW2 += dy h^T  (K = the 16 anchors)
#pragma unroll
            for (int j = 0; j < (kMaxO + 63) / 64; ++j) {
                const int m = lane + 64 * j;
                if (m < O) {
                    float sacc = 0.0f;
#pragma unroll
                    for (int al = 0; al < 16; ++al) sacc += dys[wave][al][m];
                    accB2[j] += sacc;
                }
            }
#pragma unroll
            for (int ks = 0; ks < 4; ++ks) {
                const int al = ks * 4 + (lane >> 4);
                const float hb0 = hs[wave][al][lane & 15];
                const float hb1 = hs[wave][al][16 + (lane & 15)];
#pragma unroll
                for (int t = 0; t < OT; ++t) {
                    const int m = t * 16 + (lane & 15);
                    const float av = m < O ? dys[wave][al][m] : 0.0f;
                    accW2[t][0] = mfma4(av, hb0, accW2[t][0]);
                    accW2[t][1] = mfma4(av, hb1, accW2[t][1]);
                }
            }
            // dh = W2^T dy  (K = m)
            v4f dh[2] = {v4f{0.f, 0.f, 0.f, 0.f}, v4f{0.f, 0.f, 0.f, 0.f}};
#pragma unroll
            for (int ks = 0; ks < OT * 4; ++ks) {
                const int m = ks * 4 + (lane >> 4);
                const float bv = m < O ? dys[wave][lane & 15][m] : 0.0f;
                const float* wr = w2s + (ks * 4 + (lane >> 4)) * kW2S + (lane & 15);
                dh[0] = mfma4(wr[0], bv, dh[0]);
                dh[1] = mfma4(wr[16], bv, dh[1]);
            }
            float dpre[2][4];
#pragma unroll
            for (int mt = 0; mt < 2; ++mt)
#pragma unroll
                for (int i = 0; i < 4; ++i) dpre[mt][i] = (avalid && pre[mt][i] > 0.0f) ? dh[mt][i] : 0.0f;
            // df = W1^T dpre (tile 2: the view inputs)
            v4f df[3] = {v4f{0.f, 0.f, 0.f, 0.f}, v4f{0.f, 0.f, 0.f, 0.f}, v4f{0.f, 0.f, 0.f, 0.f}};
#pragma unroll
            for (int st = 0; st < 8; ++st) {
                const float* wr = w1s + ((st >> 2) * 16 + 4 * (lane >> 4) + (st & 3)) * kW1S + (lane & 15);
                df[0] = mfma4(wr[0], dpre[st >> 2][st & 3], df[0]);
                df[1] = mfma4(wr[16], dpre[st >> 2][st & 3], df[1]);
                if (view) df[2] = mfma4(wr[32], dpre[st >> 2][st & 3], df[2]);
            }
            if (view) {  // uniform
                float dc[3] = {0.0f, 0.0f, 0.0f};  // this anchor's share of dL/d camera centre
                if (lane < 16 && avalid) {
                    // lanes 0-15 hold rows 32..35 (dL/d distance, dL/d direction) of anchor `lane`:
                    // dL/dv = dL/ddelta d + (dL/dd - (dL/dd . d) d) / delta,  v = x_a - x_c
                    const float dist = vs[wave][lane][0];
                    const float d0 = vs[wave][lane][1], d1v = vs[wave][lane][2], d2 = vs[wave][lane][3];
                    const float gd = df[2][1] * d0 + df[2][2] * d1v + df[2][3] * d2;
                    const float dv[3] = {df[2][0] * d0 + (df[2][1] - gd * d0) / dist,
                                         df[2][0] * d1v + (df[2][2] - gd * d1v) / dist,
                                         df[2][0] * d2 + (df[2][3] - gd * d2) / dist};
#pragma unroll
                    for (int i = 0; i < 3; ++i) {
                        if (out.xa) out.xa[i * a.na + an] += dv[i];
                        dc[i] = -dv[i];
                    }
                }
                // the 16 anchors' sum (lanes 0-15), added to this wave's view-v total
#pragma unroll
                for (int i = 0; i < 3; ++i)
#pragma unroll
                    for (int o = 8; o > 0; o >>= 1) dc[i] += __shfl_xor(dc[i], o, 16);
                if (lane == 0) {
#pragma unroll
                    for (int i = 0; i < 3; ++i) camw[wave][v * 3 + i] += dc[i];
                }
            }
            if (out.feat && avalid) {
#pragma unroll
                for (int ft = 0; ft < 2; ++ft)
#pragma unroll
                    for (int i = 0; i < 4; ++i) put(out.feat + an * kF + ft * 16 + 4 * (lane >> 4) + i, first, df[ft][i]);
            }
            // dW1 += dpre f^T, db1 += sum dpre (K = the 16 anchors)
#pragma unroll
            for (int mt = 0; mt < 2; ++mt)
#pragma unroll
                for (int i = 0; i < 4; ++i) ps[wave][lane & 15][mt * 16 + 4 * (lane >> 4) + i] = dpre[mt][i];
            wsync();
            if (lane < kF) {
                float sacc = 0.0f;
#pragma unroll
                for (int al = 0; al < 16; ++al) sacc += ps[wave][al][lane];
                accB1 += sacc;
            }
#pragma unroll
            for (int ks = 0; ks < 4; ++ks) {
                const int al = ks * 4 + (lane >> 4);
                const int64_t anc = a0 + al;
                const float f0 = anc < a.na ? a.feat[anc * kF + (lane & 15)] : 0.0f;
                const float f1 = anc < a.na ? a.feat[anc * kF + 16 + (lane & 15)] : 0.0f;
                const float f2 = (view && (lane & 15) < 4) ? vs[wave][al][lane & 15] : 0.0f;
#pragma unroll
                for (int nt = 0; nt < 2; ++nt) {
                    const float av = ps[wave][al][nt * 16 + (lane & 15)];
                    accW1[nt][0] = mfma4(av, f0, accW1[nt][0]);
                    accW1[nt][1] = mfma4(av, f1, accW1[nt][1]);
                    if (view) accW1[nt][2] = mfma4(av, f2, accW1[nt][2]);
                }
            }
            wsync();
        }
    }
    // block reduction in wave order, then one partial row per block
    __syncthreads();
    float* red = smem;  // bwd_smem_floats(OT) >= bwd_red_floats(OT)
    // Wave w adds the sum of waves 0..w-1 into its accumulators, then stores
    // them: all its loads are issued before any store.
    for (int w = 0; w < kBwdWaves; ++w) {
        if (wave == w) {
            if (w > 0) {
#pragma unroll
                for (int t = 0; t < OT; ++t)
#pragma unroll
                    for (int nt = 0; nt < 2; ++nt)
#pragma unroll
                        for (int i = 0; i < 4; ++i)
                            accW2[t][nt][i] += red[(t * 16 + 4 * (lane >> 4) + i) * kF + nt * 16 + (lane & 15)];
#pragma unroll
                for (int j = 0; j < (kMaxO + 63) / 64; ++j) accB2[j] += red[red_b2(OT) + lane + 64 * j];
#pragma unroll
                for (int nt = 0; nt < 2; ++nt)
#pragma unroll
                    for (int ft = 0; ft < 3; ++ft)
#pragma unroll
                        for (int i = 0; i < 4; ++i)
                            accW1[nt][ft][i] +=
                                red[red_w1(OT) + (nt * 16 + 4 * (lane >> 4) + i) * kRedW1Cols + ft * 16 + (lane & 15)];
                accB1 += red[red_b1(OT) + lane];
            }
#pragma unroll
            for (int t = 0; t < OT; ++t)
#pragma unroll
                for (int nt = 0; nt < 2; ++nt)
#pragma unroll
                    for (int i = 0; i < 4; ++i)
                        red[(t * 16 + 4 * (lane >> 4) + i) * kF + nt * 16 + (lane & 15)] = accW2[t][nt][i];
#pragma unroll
            for (int j = 0; j < (kMaxO + 63) / 64; ++j) red[red_b2(OT) + lane + 64 * j] = accB2[j];
#pragma unroll
            for (int nt = 0; nt < 2; ++nt)
#pragma unroll
                for (int ft = 0; ft < 3; ++ft)
#pragma unroll
                    for (int i = 0; i < 4; ++i)
                        red[red_w1(OT) + (nt * 16 + 4 * (lane >> 4) + i) * kRedW1Cols + ft * 16 + (lane & 15)] =
                            accW1[nt][ft][i];
            red[red_b1(OT) + lane] = accB1;
        }
        __syncthreads();
    }
    if (threadIdx.x < 3 * a.views) {  // camera-centre sums in wave order
        float c = camw[0][threadIdx.x];
        for (int w = 1; w < kBwdWaves; ++w) c += camw[w][threadIdx.x];
        red[red_cam(OT) + threadIdx.x] = c;
    }
    __syncthreads();
    // compact partial row: dW2 [O][32] | db2 [O] | dW1 [32][in_dim] | db1 [32] | dcam [views][3]
    const int64_t PF = decode_bwd_partial_floats(a.k, a.in_dim, a.views);
    const int oB2 = O * kF, oW1 = oB2 + O, oB1 = oW1 + kF * a.in_dim, oCam = oB1 + kF;
    for (int i = threadIdx.x; i < PF; i += blockDim.x) {
        int src;
        if (i < oB2) src = i;
        else if (i < oW1) src = red_b2(OT) + (i - oB2);
        else if (i < oB1) {
            const int j = i - oW1, nn = j / a.in_dim;
            src = red_w1(OT) + nn * kRedW1Cols + (j - nn * a.in_dim);
        } else if (i < oCam) src = red_b1(OT) + (i - oB1);
        else src = red_cam(OT) + (i - oCam);
        partial[blockIdx.x * PF + i] = red[src];
    }
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
