// Front-to-back compositing of colour, depth and silhouette (paper eqs. (16)-(18))
// and its replaying adjoint.
//
// Footprint of Gaussian i at pixel centre p (eq. (1) on the image plane):
//   d = p - (u, v),  alpha = min(0.99, o exp(-1/2 d^T Q d)), skipped when alpha < 1/255,
// with Q = (Sigma' + 0.3 I)^-1 held in eigen form (see Splat): the exponent is a sum
// of two non-negative terms, accurate in FP32 even for very thin footprints.
// The Gaussian whose inclusion would take the transmittance below 1e-4 is
// excluded and the pixel stops.
//
// Work layout: one wave64 per (16x16 tile, slice); a wave covers 64 * PPL
// pixels (an 8x8 quadrant at one pixel per lane; 16 wide with PPL pixels per
// lane stacked 4 rows apart otherwise) and walks its tile's
// depth-sorted list independently of the other waves.  Records are staged 64
// at a time in a wave-private LDS slab; while staging, each lane tests its own
// Gaussian's 1/255 ellipse against the wave's pixel rectangle (exact minimum of
// the quadratic form over the rectangle, with a safety margin), and the wave
// then visits only the entries that can reach one of its pixels -- entries it
// skips could only have produced alpha < 1/255, so results are unchanged.  The
// wave leaves as soon as all its pixels have stopped.  No block-wide barriers.
// Blocks are remapped so that consecutive tiles share an XCD (and its L2).
//
// Backward: the same walk in reverse, from each pixel's final transmittance and
// last contributor (saved by the forward), recovering T_i = T_{i+1} / (1 - alpha_i)
// and, instead of the normalised colour behind i, its product U with the
// pixel's upstream gradient.  The ten per-Gaussian sums are reduce-scattered
// over the wave (lane swaps across rows, DPP inside rows), parked in LDS for six
// Gaussians and added to the Gaussian's gradient slot with one atomic per value.
#include "internal.h"

namespace vcgs {

struct Fp {
    float alpha, G;
    bool clamped;
    float p1, p2;
};

// Shared by forward and backward so both take identical skip decisions.
// (ax, ay) = s1 e and (bx, by) = s2 e (see Splat): p1, p2 here are the scaled
// eigen-frame offsets q1 = s1 d . e and q2 = s2 d . e_perp, and the base-2
// exponent is -(q1^2 + q2^2).
__device__ __forceinline__ Fp footprint(float dx, float dy, float ax, float ay, float bx, float by, float o)
{
#pragma clang fp contract(off)
    Fp f;
    f.p1 = __builtin_fmaf(dy, ay, dx * ax);
    f.p2 = __builtin_fmaf(dy, bx, -(dx * by));
    const float pw = __builtin_fmaf(-f.p1, f.p1, -(f.p2 * f.p2));
    f.G = __builtin_amdgcn_exp2f(pw);
    const float raw = o * f.G;
    f.clamped = raw > kAlphaMax;
    f.alpha = fminf(raw, kAlphaMax);
    return f;
}

// Can the Gaussian reach alpha >= 1/255 at some point of [x0, x1] x [y0, y1]?
// Exact minimum of q(d) = q1^2 + q2^2 (base-2 units) over the rectangle,
// compared with log2(255 o) plus a margin far above FP32 error.  With the
// scaled rows (ax, ay) = s1 e and (bx, by) = s2 e, q(d) = A dx^2 + 2 B dx dy
// + C dy^2 with A = ax^2 + by^2, B = ax ay - bx by, C = ay^2 + bx^2.
__device__ __forceinline__ bool reaches_rect(const Splat& s, float x0, float x1, float y0, float y1)
{
    const float u = s.a.x + s.a.z, v = s.a.y + s.a.w, o = s.c.x;
    const float ax = s.b.x, ay = s.b.y, bx = s.b.z, by = s.b.w;
    const float A = ax * ax + by * by;
    const float B = ax * ay - bx * by;
    const float C = ay * ay + bx * bx;
    const float thr = __log2f(255.0f * o) * 1.001f + 1e-3f;
    if (u >= x0 && u <= x1 && v >= y0 && v <= y1) return true;
    // the edge minimisers need not be exact: any point of an edge bounds the
    // minimum from above, and a 1-ulp error moves q far less than the margin
    const float iA = __builtin_amdgcn_rcpf(A), iC = __builtin_amdgcn_rcpf(C);
    const float dx0 = x0 - u, dx1 = x1 - u, dy0 = y0 - v, dy1 = y1 - v;
    float best = 3.0e38f;
    // vertical edges: dx fixed, minimise over dy
    {
        const float dx = dx0;
        const float dy = fminf(fmaxf(-B * dx * iC, dy0), dy1);
        best = fminf(best, A * dx * dx + 2.0f * B * dx * dy + C * dy * dy);
    }
    {
        const float dx = dx1;
        const float dy = fminf(fmaxf(-B * dx * iC, dy0), dy1);
        best = fminf(best, A * dx * dx + 2.0f * B * dx * dy + C * dy * dy);
    }
    // horizontal edges: dy fixed, minimise over dx
    {
        const float dy = dy0;
        const float dx = fminf(fmaxf(-B * dy * iA, dx0), dx1);
        best = fminf(best, A * dx * dx + 2.0f * B * dx * dy + C * dy * dy);
    }
    {
        const float dy = dy1;
        const float dx = fminf(fmaxf(-B * dy * iA, dx0), dx1);
        best = fminf(best, A * dx * dx + 2.0f * B * dx * dy + C * dy * dy);
    }
    return best <= thr;
}

__device__ __forceinline__ int xcd_remap(int b, int nb)
{
    const int q = nb >> 3, r = nb & 7;
    const int x = b & 7, s = b >> 3;
    return (x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q) + s;
}

__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// View of a global tile id (views are laid out tile-major in id order).
__device__ __forceinline__ int view_of(const ViewTab& tab, uint32_t t)
{
    int v = 0;
    while (v + 1 < tab.n_views && t >= tab.tile_end[v]) ++v;
    return v;
}

template <int PPL, bool COUNT>
__global__ void __launch_bounds__(256) k_composite_fwd(ViewTab tab, uint32_t total_tiles,
                                                       const Splat* __restrict__ rec,
                                                       const uint32_t* __restrict__ gids,
                                                       const uint32_t* __restrict__ ranges,
                                                       unsigned long long* __restrict__ counters, int cull, int sched)
{
    constexpr int WPT = 4 / PPL;     // waves per tile
    constexpr int SW = PPL == 1 ? 8 : 16;  // width of a wave's pixel block (8x8 quadrants at 1 pixel per lane)
    constexpr int LR = 64 / SW;            // rows of lanes
    constexpr int SH = LR * PPL;           // height of a wave's pixel block
    // splat records staged component-major (conflict-free stores, broadcast
    // reads): rows (u, v, u_lo, v_lo), scaled eigen rows, (opacity, r, g, b),
    // (depth, Gaussian id as bits, -, -), so that every read of entry k is at a
    // fixed offset from its first row
    __shared__ float4 slab[4][4][64];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (tab.flags_out && blockIdx.x == 0 && threadIdx.x == 0) {
        tab.flags_out[0] = tab.flags_src[0];
        tab.flags_out[1] = tab.flags_src[1];
    }
    const int gw = (sched ? xcd_remap(blockIdx.x, gridDim.x) : (int)blockIdx.x) * 4 + wave;
    const uint32_t gt = (uint32_t)(gw / WPT);
    const int sub = gw % WPT;
    if (gt >= total_tiles) return;
    const int vw = view_of(tab, gt);
    const CamK& cam = tab.cam[vw];
    const int tile = (int)(gt - cam.tile_base);
    uint32_t* __restrict__ hits = tab.hits;  // uniform
    float* __restrict__ color = tab.color[vw];
    float* __restrict__ depth = tab.depth[vw];
    float* __restrict__ alpha_out = tab.alpha[vw];
    float* __restrict__ t_final = tab.t_final[vw];
    uint32_t* __restrict__ n_contrib = tab.n_contrib[vw];
    const float bg0 = tab.bg[0], bg1 = tab.bg[1], bg2 = tab.bg[2];
    uint32_t n_eval = 0, n_blend = 0;
    const int tx = tile % cam.tiles_x, ty = tile / cam.tiles_x;
    const int qx = PPL == 1 ? (sub & 1) : 0, qy = PPL == 1 ? (sub >> 1) : sub;
    const int px = tx * kTile + qx * SW + lane % SW;
    const int row0 = ty * kTile + qy * SH;
    // pixel-centre rectangle of this wave
    const float rx0 = (float)(tx * kTile + qx * SW) + 0.5f, rx1 = rx0 + (float)(SW - 1);
    const float ry0 = (float)row0 + 0.5f, ry1 = ry0 + (float)(SH - 1);
    // T < 0 marks a pixel that has stopped (or lies outside the image); |T| is
    // then its final transmittance.  Keeping the state in the sign lets the
    // blend below run without any per-lane branch or mask bookkeeping.
    float dy[PPL];
    // the silhouette sum_i alpha_i T_i telescopes to 1 - T_final: no channel of its own
    float T[PPL], c0[PPL], c1[PPL], c2[PPL], dd[PPL];
    uint32_t last[PPL];
#pragma unroll
    for (int j = 0; j < PPL; ++j) {
        const int py = row0 + lane / SW + LR * j;
        dy[j] = (float)py + 0.5f;
        T[j] = (px < cam.W && py < cam.H) ? 1.0f : -1.0f;
        c0[j] = c1[j] = c2[j] = dd[j] = 0.0f;
        last[j] = 0u;
    }
    const float pxf = (float)px + 0.5f;
    // the tile's list (wave-uniform: list positions and indices stay scalar)
    const uint32_t start = __builtin_amdgcn_readfirstlane(ranges[2 * gt]);
    const uint32_t end = __builtin_amdgcn_readfirstlane(ranges[2 * gt + 1]);
    // One footprint blended front to back into pixel j.  A Gaussian below
    // 1/255 takes alpha 0, which leaves T (>= 1e-4 while running) unchanged;
    // one that would take T below 1e-4 stops the pixel with weight 0; a stopped
    // pixel (T < 0) gets Tn <= 0 and so stays stopped with weight 0.
    auto blend = [&](int j, const Fp& f, const float4& rc, float rz, uint32_t idx, bool en) -> bool {
        const float a = (en && f.alpha >= kAlphaMin) ? f.alpha : 0.0f;
        const float Tn = T[j] * (1.0f - a);
        const bool stop = Tn < kTMin;
        const float w = stop ? 0.0f : a * T[j];
        if (COUNT) { n_eval += (en && T[j] > 0.0f) ? 1u : 0u; n_blend += w > 0.0f ? 1u : 0u; }
        c0[j] += w * rc.y; c1[j] += w * rc.z; c2[j] += w * rc.w;
        dd[j] += w * rz;
        last[j] = w > 0.0f ? idx : last[j];
        T[j] = stop ? -fabsf(T[j]) : Tn;
        return w > 0.0f;
    };
    // pixels of the wave that blended Gaussian slot k, added to its hit count
    auto add_hits = [&](int k, uint32_t nh) {
        if (lane == 0 && nh) atomicAdd(hits + __float_as_uint(slab[wave][3][k].y) % (uint32_t)tab.n, nh);
    };
    auto wave_done = [&]() {
        bool mine = true;
#pragma unroll
        for (int j = 0; j < PPL; ++j) mine = mine && T[j] < 0.0f;
        return __all(mine);
    };
    bool all_done = wave_done();  // e.g. rows below the image
    for (uint32_t b = start; b < end && !all_done; b += 64) {
        wave_lds_sync();
        const uint32_t idx = b + lane;
        bool keep = false;
        if (idx < end) {
            const uint32_t e = gids[idx];
            const Splat sp = rec[e];
            keep = !cull || reaches_rect(sp, rx0, rx1, ry0, ry1);
            slab[wave][0][lane] = sp.a;
            slab[wave][1][lane] = sp.b;
            slab[wave][2][lane] = sp.c;
            slab[wave][3][lane] = make_float4(sp.d.x, __uint_as_float(e), 0.0f, 0.0f);
        }
        uint64_t todo = __ballot(keep);
        wave_lds_sync();
        const uint32_t base = b - start + 1u;
        // two Gaussians per round: both footprints are independent, the blends are in order
        while (todo) {
            const int k1 = __builtin_ctzll(todo);
            todo &= todo - 1ull;
            const bool two = todo != 0ull;
            const int k2 = two ? __builtin_ctzll(todo) : k1;
            todo &= todo - 1ull;
            const float4 a1 = slab[wave][0][k1], b1 = slab[wave][1][k1], r1 = slab[wave][2][k1];
            const float z1 = slab[wave][3][k1].x;
            const float4 a2 = slab[wave][0][k2], b2 = slab[wave][1][k2], r2 = slab[wave][2][k2];
            const float z2 = slab[wave][3][k2].x;
            const float dx1 = (pxf - a1.x) - a1.z, dx2 = (pxf - a2.x) - a2.z;
            uint32_t h1 = 0u, h2 = 0u;
#pragma unroll
            for (int j = 0; j < PPL; ++j) {
                const Fp f1 = footprint(dx1, (dy[j] - a1.y) - a1.w, b1.x, b1.y, b1.z, b1.w, r1.x);
                const Fp f2 = footprint(dx2, (dy[j] - a2.y) - a2.w, b2.x, b2.y, b2.z, b2.w, r2.x);
                const bool t1 = blend(j, f1, r1, z1, base + (uint32_t)k1, true);
                const bool t2 = blend(j, f2, r2, z2, base + (uint32_t)k2, two);
                if (hits) {
                    h1 += (uint32_t)__popcll(__ballot(t1));
                    h2 += (uint32_t)__popcll(__ballot(t2));
                }
            }
            if (hits) {
                add_hits(k1, h1);
                if (two) add_hits(k2, h2);
            }
            if (wave_done()) { all_done = true; break; }
        }
    }
#pragma unroll
    for (int j = 0; j < PPL; ++j) T[j] = fabsf(T[j]);
    const int HW = cam.W * cam.H;
#pragma unroll
    for (int j = 0; j < PPL; ++j) {
        const int py = row0 + lane / SW + LR * j;
        if (px < cam.W && py < cam.H) {
            const int p = py * cam.W + px;
            color[p] = c0[j] + T[j] * bg0;
            color[HW + p] = c1[j] + T[j] * bg1;
            color[2 * HW + p] = c2[j] + T[j] * bg2;
            depth[p] = dd[j];
            alpha_out[p] = 1.0f - T[j];
            if (t_final) {  // null for forward-only callers
                t_final[p] = T[j];
                n_contrib[p] = last[j];
            }
        }
    }
    if (COUNT) {
        if (n_eval) atomicAdd(counters + 0, (unsigned long long)n_eval);
        if (n_blend) atomicAdd(counters + 1, (unsigned long long)n_blend);
    }
}

// Sum over the 64 lanes, result in every lane.
__device__ __forceinline__ float wave_sum(float v)
{
    v += __builtin_amdgcn_update_dpp(0.0f, v, 0xB1, 0xF, 0xF, false);   // quad_perm [1,0,3,2]
    v += __builtin_amdgcn_update_dpp(0.0f, v, 0x4E, 0xF, 0xF, false);   // quad_perm [2,3,0,1]
    v += __builtin_amdgcn_update_dpp(0.0f, v, 0x124, 0xF, 0xF, false);  // row_ror:4
    v += __builtin_amdgcn_update_dpp(0.0f, v, 0x128, 0xF, 0xF, false);  // row_ror:8
    const float r0 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 0));
    const float r1 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 16));
    const float r2 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 32));
    const float r3 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 48));
    return (r0 + r1) + (r2 + r3);
}

__device__ __forceinline__ uint32_t wave_max_u32(uint32_t v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = max(v, (uint32_t)__shfl_xor((int)v, o, 64));
    return v;
}

// keep + (the partner lane's send) for a DPP partner pattern within 16-lane rows.
template <int CTRL>
__device__ __forceinline__ float dpp_add(float keep, float send)
{
    return keep + __builtin_amdgcn_update_dpp(0.0f, send, CTRL, 0xF, 0xF, true);
}

// Reduce-scatter of ten per-lane values over the whole wave.  The two
// cross-row steps use the gfx950 lane swaps: v_permlane32_swap exchanges the
// upper 32 lanes of one register with the lower 32 lanes of another, so after
// one swap and one add lanes 0-31 hold value k summed over (l, l + 32) and
// lanes 32-63 value k + 5; v_permlane16_swap does the same for odd and even
// 16-lane rows.  The last four steps pair lanes inside each row with DPP
// (c^8 by row_ror:8, then the half-row mirror, then c^2 and c^1); at the c^8
// and mirror steps each lane keeps one of two values and passes the other.
// Afterwards the total of value q is in lane wr_lane(q) (and a few others):
// 26 lane operations for ten totals, no LDS.
__device__ __forceinline__ float swap_add32(float x, float y)
{
    const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(x), __float_as_uint(y), false, false);
    return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}
__device__ __forceinline__ float swap_add16(float x, float y)
{
    const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(x), __float_as_uint(y), false, false);
    return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}
__device__ __forceinline__ float wave_reduce10(const float p[10], int lane)
{
    float a[5];
#pragma unroll
    for (int k = 0; k < 5; ++k) a[k] = swap_add32(p[k], p[k + 5]);  // value k + 5 (lane & 32)
    const float b0 = swap_add16(a[0], a[1]);  // value 0 + (lane & 16 ? 1 : 0)
    const float b1 = swap_add16(a[2], a[3]);  // value 2 + (lane & 16 ? 1 : 0)
    const float b2 = swap_add16(a[4], a[4]);  // value 4, in every row
    const bool h3 = lane & 8, h2 = lane & 4;
    const float c0 = dpp_add<0x128>(h3 ? b1 : b0, h3 ? b0 : b1);
    const float c1 = dpp_add<0x128>(b2, b2);
    const float d0 = dpp_add<0x141>(h2 ? c1 : c0, h2 ? c0 : c1);
    const float e0 = dpp_add<0x4E>(d0, d0);
    return dpp_add<0xB1>(e0, e0);
}
// Which total lane `lane` holds after wave_reduce10, or -1 if it is not the
// lane that passes it on (one lane per value).
__device__ __forceinline__ int wr_value(int lane)
{
    if (lane & 3) return -1;
    const int h5 = (lane >> 5) & 1, h4 = (lane >> 4) & 1, h3 = (lane >> 3) & 1, h2 = (lane >> 2) & 1;
    if (h2) return (h3 || h4) ? -1 : 4 + 5 * h5;
    return 2 * h3 + h4 + 5 * h5;
}

// One list entry k of a staged slab for the wave's pixels (local = its index
// in the tile's list): footprints, then, if it blends into any of the wave's
// pixels, the adjoint of each pixel's blend, returned as the ten per-lane sums
// p (p0-p4: dL/dpower against the scaled eigen-frame offset (q1, q2, q1^2,
// q1 q2, q2^2), p5: dL/dopacity, p6-p9: dL/d(r, g, b, depth)), stepping T and U back
// over the entry.  Returns false (and changes nothing) when no lane blends it.
template <int PPL, bool COUNT>
__device__ __forceinline__ bool adjoint_entry(const float4* s0, const float4* s1, const float4* s2, const float* sz,
                                              int k, uint32_t local, float pxf, const float pyf[PPL],
                                              const uint32_t last[PPL], float T[PPL], float U[PPL],
                                              const float up[PPL][5], float p[10], uint32_t& n_eval,
                                              uint32_t& n_blend)
{
    const float4 ra = s0[k], rb = s1[k];
    const float dx = (pxf - ra.x) - ra.z;
    // footprints first: a wave-entry that blends into none of the wave's
    // pixels changes no state and adds nothing, so it skips the adjoint
    Fp fj[PPL];
    bool cj[PPL];
    bool any = false;
#pragma unroll
    for (int j = 0; j < PPL; ++j) {
        fj[j] = footprint(dx, (pyf[j] - ra.y) - ra.w, rb.x, rb.y, rb.z, rb.w, s2[k].x);
        const bool in = local < last[j];
        cj[j] = in && fj[j].alpha >= kAlphaMin;
        if (COUNT) { n_eval += in ? 1u : 0u; n_blend += cj[j] ? 1u : 0u; }
        any = any || cj[j];
    }
    if (__ballot(any) == 0ull) return false;
    const float4 rc = s2[k];
    const float rz = sz[k];
#pragma unroll
    for (int i = 0; i < 10; ++i) p[i] = 0.0f;
#pragma unroll
    for (int j = 0; j < PPL; ++j) {
        // branch-free: every lane evaluates, only contributing pixels change state
        const Fp& f = fj[j];
        const bool c = cj[j];
        const float a = f.alpha;
        const float Ti = T[j] * __builtin_amdgcn_rcpf(1.0f - a);
        const float X = fmaf(up[j][0], rc.y, fmaf(up[j][1], rc.z, fmaf(up[j][2], rc.w, fmaf(up[j][3], rz, up[j][4]))));
        const float d = X - U[j];
        U[j] = fmaf(c ? a : 0.0f, d, U[j]);
        const float w = c ? a * Ti : 0.0f;
        p[6] = fmaf(w, up[j][0], p[6]);
        p[7] = fmaf(w, up[j][1], p[7]);
        p[8] = fmaf(w, up[j][2], p[8]);
        p[9] = fmaf(w, up[j][3], p[9]);
        const float dg = (c && !f.clamped) ? d * Ti : 0.0f;  // dL/d(o G)
        const float dP = dg * a;                             // dL/dpower
        const float t1 = dP * f.p1, t2 = dP * f.p2;
        p[0] += t1;
        p[1] += t2;
        p[2] = fmaf(t1, f.p1, p[2]);
        p[3] = fmaf(t1, f.p2, p[3]);
        p[4] = fmaf(t2, f.p2, p[4]);
        p[5] = fmaf(dg, f.G, p[5]);
        T[j] = c ? Ti : T[j];
    }
    return true;
}

constexpr int kPend = 6;  // Gaussians whose totals are gathered before one atomic flush

template <int PPL, bool COUNT>
__global__ void __launch_bounds__(256) k_composite_bwd(ViewTab tab, uint32_t total_tiles,
                                                       const Splat* __restrict__ rec,
                                                       const uint32_t* __restrict__ gids,
                                                       const uint32_t* __restrict__ ranges, float* __restrict__ g2,
                                                       unsigned long long* __restrict__ counters, int cull, int sched)
{
    constexpr int WPT = 4 / PPL;
    constexpr int SW = PPL == 1 ? 8 : 16;
    constexpr int LR = 64 / SW;
    constexpr int SH = LR * PPL;
    // splat records staged component-major (conflict-free stores, broadcast
    // reads), rows grouped by use so that every read is at a fixed offset from
    // entry k's first row: 0 = (u, v, u_lo, v_lo), 1 = scaled eigen rows, both
    // read for every entry; 2 = (r, g, b, depth), read only for a blending
    // entry; 3 = (opacity, Gaussian id as bits, -, -)
    __shared__ float4 slab[4][4][64];
    // per-Gaussian totals (10 values) waiting to be added to g2, slot-major
    __shared__ float pend[4][kPend * 10];
    __shared__ uint32_t pend_gid[4][kPend];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int gw = (sched ? xcd_remap(blockIdx.x, gridDim.x) : (int)blockIdx.x) * 4 + wave;
    const uint32_t gt = (uint32_t)(gw / WPT);
    const int sub = gw % WPT;
    if (gt >= total_tiles) return;
    const int vw = view_of(tab, gt);
    const CamK& cam = tab.cam[vw];
    const int tile = (int)(gt - cam.tile_base);
    const float* __restrict__ t_final = tab.t_final[vw];
    const uint32_t* __restrict__ n_contrib = tab.n_contrib[vw];
    const float* __restrict__ dl_dc = tab.dl_dc[vw];
    const float* __restrict__ dl_dd = tab.dl_dd[vw];
    const float* __restrict__ dl_da = tab.dl_da[vw];
    const float bg0 = tab.bg[0], bg1 = tab.bg[1], bg2 = tab.bg[2];
    uint32_t n_eval = 0, n_blend = 0, n_flush = 0;
    int npend = 0, poff = 0;  // uniform; poff = 10 npend, kept by addition (no multiply in the address)
    const int wrv = wr_value(lane);
    float* const pend_lane = &pend[wave][wrv < 0 ? 0 : wrv];  // this lane's total, slot 0
    const int tx = tile % cam.tiles_x, ty = tile / cam.tiles_x;
    const int qx = PPL == 1 ? (sub & 1) : 0, qy = PPL == 1 ? (sub >> 1) : sub;
    const int px = tx * kTile + qx * SW + lane % SW;
    const int row0 = ty * kTile + qy * SH;
    const float rx0 = (float)(tx * kTile + qx * SW) + 0.5f, rx1 = rx0 + (float)(SW - 1);
    const float ry0 = (float)row0 + 0.5f, ry1 = ry0 + (float)(SH - 1);
    const int HW = cam.W * cam.H;
    // Per pixel: T = transmittance in front of the current entry, up = upstream
    // gradient of (r, g, b, depth, alpha), U = up . acc where acc is the
    // normalised composite behind the current entry ((bg, 0, 0) behind the
    // last one).  acc itself is never needed: dL/dalpha_i = T_i (up . x_i - U)
    // with x_i = (c_i, z_i, 1), and acc <- acc + alpha (x - acc) gives
    // U <- U + alpha (up . x - U).
    float T[PPL], up[PPL][5], U[PPL];
    uint32_t last[PPL];
    float pyf[PPL];
    uint32_t wl = 0;
#pragma unroll
    for (int j = 0; j < PPL; ++j) {
        const int py = row0 + lane / SW + LR * j;
        pyf[j] = (float)py + 0.5f;
        const bool in = px < cam.W && py < cam.H;
        const int p = py * cam.W + px;
        T[j] = in ? t_final[p] : 1.0f;
        last[j] = in ? n_contrib[p] : 0u;
        up[j][0] = (in && dl_dc) ? dl_dc[p] : 0.0f;
        up[j][1] = (in && dl_dc) ? dl_dc[HW + p] : 0.0f;
        up[j][2] = (in && dl_dc) ? dl_dc[2 * HW + p] : 0.0f;
        up[j][3] = (in && dl_dd) ? dl_dd[p] : 0.0f;
        up[j][4] = (in && dl_da) ? dl_da[p] : 0.0f;
        U[j] = fmaf(up[j][0], bg0, fmaf(up[j][1], bg1, up[j][2] * bg2));
        wl = max(wl, last[j]);
    }
    const float pxf = (float)px + 0.5f;
    wl = wave_max_u32(wl);
    if (wl == 0u) return;  // uniform across the wave
    const uint32_t start = ranges[2 * gt];
    auto flush = [&](int count) {
        wave_lds_sync();
        if (lane < 10 * count) {
            const int sl = lane / 10, v = lane - 10 * sl;
            atomicAdd(g2 + (size_t)kG2 * pend_gid[wave][sl] + v, pend[wave][lane]);
        }
        wave_lds_sync();
    };
    // rem[j] = last[j] - bs: entry k of the slab at bs lies in front of pixel
    // j's last contributor iff k < rem[j]
    int rem[PPL];
    const int bs0 = (int)((wl - 1u) & ~63u);
#pragma unroll
    for (int j = 0; j < PPL; ++j) rem[j] = (int)last[j] - bs0;
    for (int bs = bs0; bs >= 0; bs -= 64) {
        wave_lds_sync();
        const uint32_t li = (uint32_t)bs + lane;
        bool keep = false;
        if (li < wl) {
            const uint32_t g = gids[start + li];
            const Splat sp = rec[g];
            keep = !cull || reaches_rect(sp, rx0, rx1, ry0, ry1);
            slab[wave][0][lane] = sp.a;
            slab[wave][1][lane] = sp.b;
            slab[wave][2][lane] = make_float4(sp.c.y, sp.c.z, sp.c.w, sp.d.x);
            slab[wave][3][lane] = make_float4(sp.c.x, __uint_as_float(g), 0.0f, 0.0f);
        }
        uint64_t hits = __ballot(keep);
        wave_lds_sync();
        while (hits) {
            const int k = 63 - __builtin_clzll(hits);
            hits &= ~(1ull << k);
            const float4 ra = slab[wave][0][k], rb = slab[wave][1][k];
            const float dx = (pxf - ra.x) - ra.z;
            // footprints first: a wave-entry that blends into none of the wave's
            // pixels changes no state and adds nothing, so it skips the adjoint
            Fp fj[PPL];
            bool cj[PPL];
            bool any = false;
#pragma unroll
            for (int j = 0; j < PPL; ++j) {
                fj[j] = footprint(dx, (pyf[j] - ra.y) - ra.w, rb.x, rb.y, rb.z, rb.w, slab[wave][3][k].x);
                const bool in = k < rem[j];
                cj[j] = in && fj[j].alpha >= kAlphaMin;
                if (COUNT) { n_eval += in ? 1u : 0u; n_blend += cj[j] ? 1u : 0u; }
                any = any || cj[j];
            }
            if (__ballot(any) == 0ull) continue;
            const float4 rc = slab[wave][2][k];  // (r, g, b, depth)
            // Per-lane sums: p0 = sum dP q1, p1 = sum dP q2, p2 = sum dP q1^2,
            // p3 = sum dP q1 q2, p4 = sum dP q2^2 (dP = dL/dpower, (q1, q2) the
            // scaled pixel offset in the footprint's eigen frame; the projection
            // adjoint turns them into dL/d(u, v) and dL/d(conic)), p5 = dL/dopacity,
            // p6-p9 = dL/d(r, g, b, depth).
            float p[10];
#pragma unroll
            for (int i = 0; i < 10; ++i) p[i] = 0.0f;
#pragma unroll
            for (int j = 0; j < PPL; ++j) {
                // branch-free: every lane evaluates, only contributing pixels change state
                const Fp& f = fj[j];
                const bool c = cj[j];
                const float a = f.alpha;
                const float Ti = T[j] * __builtin_amdgcn_rcpf(1.0f - a);
                const float X = fmaf(up[j][0], rc.x, fmaf(up[j][1], rc.y, fmaf(up[j][2], rc.z, fmaf(up[j][3], rc.w, up[j][4]))));
                const float d = X - U[j];
                U[j] = fmaf(c ? a : 0.0f, d, U[j]);
                const float w = c ? a * Ti : 0.0f;
                p[6] = fmaf(w, up[j][0], p[6]);
                p[7] = fmaf(w, up[j][1], p[7]);
                p[8] = fmaf(w, up[j][2], p[8]);
                p[9] = fmaf(w, up[j][3], p[9]);
                const float dg = (c && !f.clamped) ? d * Ti : 0.0f;  // dL/d(o G)
                const float dP = dg * a;                             // dL/dpower
                const float t1 = dP * f.p1, t2 = dP * f.p2;
                p[0] += t1;
                p[1] += t2;
                p[2] = fmaf(t1, f.p1, p[2]);
                p[3] = fmaf(t1, f.p2, p[3]);
                p[4] = fmaf(t2, f.p2, p[4]);
                p[5] = fmaf(dg, f.G, p[5]);
                T[j] = c ? Ti : T[j];
            }
            const float tot = wave_reduce10(p, lane);
            if (wrv >= 0) pend_lane[poff] = tot;
            if (lane == 0) pend_gid[wave][npend] = __float_as_uint(slab[wave][3][k].y);
            ++npend;
            poff += 10;
            if (COUNT && lane == 0) ++n_flush;
            if (npend == kPend) {
                flush(kPend);
                npend = 0;
                poff = 0;
            }
        }
#pragma unroll
        for (int j = 0; j < PPL; ++j) rem[j] += 64;
    }
    if (npend > 0) flush(npend);
    if (COUNT) {
        if (n_eval) atomicAdd(counters + 2, (unsigned long long)n_eval);
        if (n_blend) atomicAdd(counters + 3, (unsigned long long)n_blend);
        if (n_flush) atomicAdd(counters + 4, (unsigned long long)n_flush);
    }
}

// The backward with the four waves of a tile (one pixel per lane: 8x8
// quadrants) in step, one slab of 64 list entries at a time: the slab's
// records are staged once for the block, every wave adds its per-Gaussian
// totals (after its own reduce-scatter) into the slab's LDS accumulator, and
// after the slab the block adds the nonzero totals to g2, one atomic per value:
// one flush per (tile, Gaussian) instead of one per (quadrant, Gaussian).
template <bool COUNT>
__global__ void __launch_bounds__(256) k_composite_bwd_tile(ViewTab tab, uint32_t total_tiles,
                                                            const Splat* __restrict__ rec,
                                                            const uint32_t* __restrict__ gids,
                                                            const uint32_t* __restrict__ ranges,
                                                            float* __restrict__ g2,
                                                            unsigned long long* __restrict__ counters, int cull,
                                                            int sched)
{
    __shared__ float4 slab[3][64];
    __shared__ float slab_z[64];
    __shared__ uint32_t slab_gid[64];
    __shared__ float acc[64][11];  // 10 totals per entry (one spare word against bank conflicts)
    __shared__ uint32_t s_wl[4];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const uint32_t gt = (uint32_t)(sched ? xcd_remap(blockIdx.x, gridDim.x) : (int)blockIdx.x);
    if (gt >= total_tiles) return;  // uniform across the block
    const int vw = view_of(tab, gt);
    const CamK& cam = tab.cam[vw];
    const int tile = (int)(gt - cam.tile_base);
    const float* __restrict__ t_final = tab.t_final[vw];
    const uint32_t* __restrict__ n_contrib = tab.n_contrib[vw];
    const float* __restrict__ dl_dc = tab.dl_dc[vw];
    const float* __restrict__ dl_dd = tab.dl_dd[vw];
    const float* __restrict__ dl_da = tab.dl_da[vw];
    uint32_t n_eval = 0, n_blend = 0, n_flush = 0;
    const int wrv = wr_value(lane);
    const int tx = tile % cam.tiles_x, ty = tile / cam.tiles_x;
    const int px = tx * kTile + (wave & 1) * 8 + (lane & 7);
    const int py = ty * kTile + (wave >> 1) * 8 + (lane >> 3);
    const float rx0 = (float)(tx * kTile + (wave & 1) * 8) + 0.5f, rx1 = rx0 + 7.0f;
    const float ry0 = (float)(ty * kTile + (wave >> 1) * 8) + 0.5f, ry1 = ry0 + 7.0f;
    const int HW = cam.W * cam.H;
    const bool in = px < cam.W && py < cam.H;
    const int pix = py * cam.W + px;
    float T[1], up[1][5], U[1];
    uint32_t last[1];
    const float pyf[1] = {(float)py + 0.5f};
    T[0] = in ? t_final[pix] : 1.0f;
    last[0] = in ? n_contrib[pix] : 0u;
    up[0][0] = (in && dl_dc) ? dl_dc[pix] : 0.0f;
    up[0][1] = (in && dl_dc) ? dl_dc[HW + pix] : 0.0f;
    up[0][2] = (in && dl_dc) ? dl_dc[2 * HW + pix] : 0.0f;
    up[0][3] = (in && dl_dd) ? dl_dd[pix] : 0.0f;
    up[0][4] = (in && dl_da) ? dl_da[pix] : 0.0f;
    U[0] = fmaf(up[0][0], tab.bg[0], fmaf(up[0][1], tab.bg[1], up[0][2] * tab.bg[2]));
    const float pxf = (float)px + 0.5f;
    const uint32_t wl = wave_max_u32(last[0]);
    if (lane == 0) s_wl[wave] = wl;
    for (int i = threadIdx.x; i < 64 * 11; i += 256) (&acc[0][0])[i] = 0.0f;
    __syncthreads();
    const uint32_t bwl = max(max(s_wl[0], s_wl[1]), max(s_wl[2], s_wl[3]));
    const uint32_t start = ranges[2 * gt];
    for (int bs = bwl ? (int)((bwl - 1u) & ~63u) : -1; bs >= 0; bs -= 64) {  // uniform across the block
        {
            // stage: thread t loads quarter t / 64 of record t % 64
            const int r = threadIdx.x & 63, q = threadIdx.x >> 6;
            const uint32_t li = (uint32_t)bs + r;
            if (li < bwl) {
                const uint32_t g = gids[start + li];
                const float4 v = reinterpret_cast<const float4*>(rec + g)[q];
                if (q < 3) slab[q][r] = v; else slab_z[r] = v.x;
                if (q == 0) slab_gid[r] = g;
            }
        }
        __syncthreads();
        // this wave's entries of the slab: below its own last contributor and
        // (with culling) reaching its quadrant
        bool keep = false;
        if ((uint32_t)bs + lane < wl) {
            Splat sp;
            sp.a = slab[0][lane];
            sp.b = slab[1][lane];
            sp.c = slab[2][lane];
            keep = !cull || reaches_rect(sp, rx0, rx1, ry0, ry1);
        }
        uint64_t hits = __ballot(keep);
        while (hits) {
            const int k = 63 - __builtin_clzll(hits);
            hits &= ~(1ull << k);
            float p[10];
            if (!adjoint_entry<1, COUNT>(slab[0], slab[1], slab[2], slab_z, k, (uint32_t)(bs + k), pxf, pyf, last, T,
                                         U, up, p, n_eval, n_blend))
                continue;
            const float tot = wave_reduce10(p, lane);
            if (wrv >= 0) atomicAdd(&acc[k][wrv], tot);
        }
        __syncthreads();
        // flush: the block's nonzero totals of the slab, one atomic per value
        for (int i = threadIdx.x; i < 64 * 10; i += 256) {
            const int k = i / 10, v = i - 10 * k;
            const float t = acc[k][v];
            if (t != 0.0f) {
                atomicAdd(g2 + (size_t)kG2 * slab_gid[k] + v, t);
                acc[k][v] = 0.0f;
                if (COUNT && v == 0) ++n_flush;
            }
        }
        __syncthreads();
    }
    if (COUNT) {
        if (n_eval) atomicAdd(counters + 2, (unsigned long long)n_eval);
        if (n_blend) atomicAdd(counters + 3, (unsigned long long)n_blend);
        if (n_flush) atomicAdd(counters + 4, (unsigned long long)n_flush);
    }
}

Options& options()
{
    static Options o;
    return o;
}

template <int PPL>
static void fwd_launch(int blocks, hipStream_t s, const ViewTab& v, uint32_t total_tiles, const Splat* rec,
                       const uint32_t* gids, const uint32_t* ranges, unsigned long long* counters, int cull,
                       int sched)
{
    if (counters)
        k_composite_fwd<PPL, true><<<blocks, 256, 0, s>>>(v, total_tiles, rec, gids, ranges, counters, cull, sched);
    else
        k_composite_fwd<PPL, false><<<blocks, 256, 0, s>>>(v, total_tiles, rec, gids, ranges, nullptr, cull, sched);
}

template <int PPL>
static void bwd_launch(int blocks, hipStream_t s, const ViewTab& v, uint32_t total_tiles, const Splat* rec,
                       const uint32_t* gids, const uint32_t* ranges, float* g2, unsigned long long* counters, int cull,
                       int sched)
{
    if (counters)
        k_composite_bwd<PPL, true><<<blocks, 256, 0, s>>>(v, total_tiles, rec, gids, ranges, g2, counters, cull,
                                                           sched);
    else
        k_composite_bwd<PPL, false><<<blocks, 256, 0, s>>>(v, total_tiles, rec, gids, ranges, g2, nullptr, cull,
                                                            sched);
}

void launch_composite_fwd(const ViewTab& v, uint32_t total_tiles, const Splat* rec, const uint32_t* gids,
                          const uint32_t* ranges, unsigned long long* counters, hipStream_t s)
{
    if (total_tiles == 0) return;
    const int ppl = options().ppl_fwd, cull = options().cull, sched = options().sched;
    const int blocks = (int)(((int64_t)total_tiles * (4 / ppl) + 3) / 4);
    if (ppl == 4) fwd_launch<4>(blocks, s, v, total_tiles, rec, gids, ranges, counters, cull, sched);
    else if (ppl == 2) fwd_launch<2>(blocks, s, v, total_tiles, rec, gids, ranges, counters, cull, sched);
    else fwd_launch<1>(blocks, s, v, total_tiles, rec, gids, ranges, counters, cull, sched);
}

void launch_composite_bwd(const ViewTab& v, uint32_t total_tiles, const Splat* rec, const uint32_t* gids,
                          const uint32_t* ranges, float* g2, unsigned long long* counters, hipStream_t s)
{
    if (total_tiles == 0) return;
    const int ppl = options().ppl_bwd, cull = options().cull, sched = options().sched;
    if (ppl == 1 && options().bwd_merge) {  // one block per tile, the waves' totals merged per slab
        if (counters)
            k_composite_bwd_tile<true><<<total_tiles, 256, 0, s>>>(v, total_tiles, rec, gids, ranges, g2, counters,
                                                                    cull, sched);
        else
            k_composite_bwd_tile<false><<<total_tiles, 256, 0, s>>>(v, total_tiles, rec, gids, ranges, g2, nullptr,
                                                                     cull, sched);
        return;
    }
    const int blocks = (int)(((int64_t)total_tiles * (4 / ppl) + 3) / 4);
    if (ppl == 4) bwd_launch<4>(blocks, s, v, total_tiles, rec, gids, ranges, g2, counters, cull, sched);
    else if (ppl == 2) bwd_launch<2>(blocks, s, v, total_tiles, rec, gids, ranges, g2, counters, cull, sched);
    else bwd_launch<1>(blocks, s, v, total_tiles, rec, gids, ranges, g2, counters, cull, sched);
}

// L1 loss: L = mean_p (sum_c |C - C*| + w_depth |D - D*|).  Image gradients per
// pixel; the scalar is reduced per block and then over blocks in block order.
constexpr int kLossThreads = 256;

// Sign of e scaled by g (0 at e = 0): the L1 gradient of one value.
__device__ __forceinline__ float l1_grad(float e, float g) { return e > 0.0f ? g : (e < 0.0f ? -g : 0.0f); }

// PX consecutive pixels per thread: 4 with 16-byte loads and stores (every
// plane 16-byte aligned and npix a multiple of 4), else 1.
template <int PX>
__global__ void __launch_bounds__(kLossThreads) k_l1_loss(int64_t npix, const float* __restrict__ c,
                                                          const float* __restrict__ d, const float* __restrict__ tc,
                                                          const float* __restrict__ td, float w_depth, float inv_n,
                                                          float* __restrict__ dl_dc, float* __restrict__ dl_dd,
                                                          float* __restrict__ partial)
{
    const int64_t p = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * PX;
    const float gd = w_depth * inv_n;
    float l = 0.0f;
    if (PX == 4 && p < npix) {
#pragma unroll
        for (int ch = 0; ch < 4; ++ch) {
            const float* a = ch < 3 ? c + ch * npix : d;
            const float* b = ch < 3 ? tc + ch * npix : td;
            float* o = ch < 3 ? dl_dc + ch * npix : dl_dd;
            const float g = ch < 3 ? inv_n : gd, w = ch < 3 ? 1.0f : w_depth;
            const float4 x = *reinterpret_cast<const float4*>(a + p), y = *reinterpret_cast<const float4*>(b + p);
            const float e0 = x.x - y.x, e1 = x.y - y.y, e2 = x.z - y.z, e3 = x.w - y.w;
            *reinterpret_cast<float4*>(o + p) = make_float4(l1_grad(e0, g), l1_grad(e1, g), l1_grad(e2, g), l1_grad(e3, g));
            l += w * ((fabsf(e0) + fabsf(e1)) + (fabsf(e2) + fabsf(e3)));
        }
    } else if (PX == 1 && p < npix) {
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) {
            const float e = c[ch * npix + p] - tc[ch * npix + p];
            dl_dc[ch * npix + p] = l1_grad(e, inv_n);
            l += fabsf(e);
        }
        const float e = d[p] - td[p];
        dl_dd[p] = l1_grad(e, gd);
        l += w_depth * fabsf(e);
    }
    if (partial) {
        __shared__ float ws[kLossThreads / 64];
        l = wave_sum(l);
        if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = l;
        __syncthreads();
        if (threadIdx.x == 0) partial[blockIdx.x] = (ws[0] + ws[1]) + (ws[2] + ws[3]);
    }
}

__device__ __forceinline__ void k_sum_partials_body(const float* __restrict__ partial, int n, float scale,
                                                    float* __restrict__ out)
{
    __shared__ double acc[4];
    double a[1] = {0.0};
    for (int i = threadIdx.x; i < n; i += 256) a[0] += (double)partial[i];
    block_sum_f64<1>(a, acc);
    if (threadIdx.x == 0) *out = (float)(a[0] * (double)scale);
}

__global__ void __launch_bounds__(256) k_sum_partials(const float* __restrict__ partial, int n, float scale,
                                                      float* __restrict__ out)
{
    k_sum_partials_body(partial, n, scale, out);
}

// The same loss for up to 16 views in two launches: view v owns blocks
// [block0[v], block0[v+1]) of the first and block v of the second, with the
// per-view arithmetic and summation order of the single-view launch.
__global__ void __launch_bounds__(kLossThreads) k_l1_loss_views(LossTab t, float* __restrict__ partial)
{
    int v = 0;
    while (v + 1 < t.n_views && (int)blockIdx.x >= t.block0[v + 1]) ++v;
    const int64_t npix = t.npix[v];
    const float inv_n = 1.0f / (float)npix;
    const int64_t p = (int64_t)(blockIdx.x - t.block0[v]) * kLossThreads + threadIdx.x;
    const float* __restrict__ c = t.c[v];
    const float* __restrict__ d = t.d[v];
    const float* __restrict__ tc = t.tc[v];
    const float* __restrict__ td = t.td[v];
    float l = 0.0f;
    if (p < npix) {
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) {
            const float e = c[ch * npix + p] - tc[ch * npix + p];
            t.dlc[v][ch * npix + p] = e > 0.0f ? inv_n : (e < 0.0f ? -inv_n : 0.0f);
            l += fabsf(e);
        }
        const float e = d[p] - td[p];
        t.dld[v][p] = e > 0.0f ? t.w_depth * inv_n : (e < 0.0f ? -t.w_depth * inv_n : 0.0f);
        l += t.w_depth * fabsf(e);
    }
    __shared__ float ws[kLossThreads / 64];
    l = wave_sum(l);
    if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = l;
    __syncthreads();
    if (threadIdx.x == 0) partial[blockIdx.x] = (ws[0] + ws[1]) + (ws[2] + ws[3]);
}

__global__ void __launch_bounds__(256) k_sum_partials_views(const float* __restrict__ partial, LossTab t,
                                                            float* __restrict__ loss)
{
    const int v = blockIdx.x;
    k_sum_partials_body(partial + t.block0[v], t.block0[v + 1] - t.block0[v], 1.0f / (float)t.npix[v], loss + v);
}

int l1_loss_blocks(int64_t npix) { return (int)((npix + kLossThreads - 1) / kLossThreads); }

void launch_l1_loss_views(const LossTab& t, float* loss, float* partial, hipStream_t s)
{
    if (t.n_views <= 0) return;
    const int nb = t.block0[t.n_views];
    if (nb > 0) k_l1_loss_views<<<nb, kLossThreads, 0, s>>>(t, partial);
    if (loss) k_sum_partials_views<<<t.n_views, 256, 0, s>>>(partial, t, loss);
}

void launch_l1_loss(int64_t npix, const float* c, const float* d, const float* tc, const float* td, float w_depth,
                    float* dl_dc, float* dl_dd, float* loss, float* partial, hipStream_t s)
{
    if (npix <= 0) {
        if (loss) launch_fill_f32(loss, 0.0f, 1, s);
        return;
    }
    const float inv_n = 1.0f / (float)npix;
    bool vec = npix % 4 == 0;
    for (const void* q : {(const void*)c, (const void*)d, (const void*)tc, (const void*)td, (const void*)dl_dc,
                          (const void*)dl_dd})
        vec = vec && (reinterpret_cast<uintptr_t>(q) & 15u) == 0u;
    // at most l1_loss_blocks(npix) partials either way
    const int nb = vec ? (int)((npix / 4 + kLossThreads - 1) / kLossThreads) : l1_loss_blocks(npix);
    float* part = loss ? partial : nullptr;
    if (vec)
        k_l1_loss<4><<<nb, kLossThreads, 0, s>>>(npix, c, d, tc, td, w_depth, inv_n, dl_dc, dl_dd, part);
    else
        k_l1_loss<1><<<nb, kLossThreads, 0, s>>>(npix, c, d, tc, td, w_depth, inv_n, dl_dc, dl_dd, part);
    if (loss) k_sum_partials<<<1, 256, 0, s>>>(partial, nb, inv_n, loss);
}

}  // namespace vcgs
