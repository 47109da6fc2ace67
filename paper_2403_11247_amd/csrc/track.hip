// Tracking and bundle-adjustment losses on the GPU (paper Sec. 3.5).
//
//   track loss   eqs. (19), (21): colour over all N = H W pixels and depth over
//                the rays with an observation (D* > 0), each pixel counted only
//                where the rendered silhouette S(p) exceeds the threshold
//                (0.99); squared errors (the paper's form) or absolute errors.
//   ICP          eq. (20): sum_i w_i |R p_i + t - q_i|^2 with q_i the nearest
//                observed point (depth back-projected at pixel centres, every
//                s-th pixel) and w_i = 1 iff that distance is below tau.
//   SSIM         the BA colour term: 1 - mean SSIM (11 x 11 Gaussian window,
//                sigma 1.5, zero padding) and its gradient.
//
// All three are HBM- or latency-bound elementwise/stencil work, so they are
// laid out for coalescing and LDS reuse rather than matrix cores.  Every sum
// is taken per block and then over blocks in block order (binary64), so the
// results are deterministic.
//
// Nearest neighbours for ICP: a point q within tau of the camera-frame centre
// x (x_z > tau) projects within f tau (1 + |x_x / x_z|) / (x_z - tau) pixels of
// x's projection along u (likewise along v), so scanning that window of the
// depth map finds exactly the nearest observed point whenever one lies within
// tau; beyond tau w = 0 and the point does not matter.  When x_z <= tau the
// bound does not hold and the window is the whole image.  Inside the window
// only the 16 x 16 tiles whose observed depth range meets (x_z - tau, x_z + tau)
// are scanned: a point of any other tile is at least tau away along z alone.
#include "internal.h"

namespace vcgs {

constexpr int kTrackThreads = 256;
constexpr int kTrackMaxBlocks = 1024;

int track_blocks(int64_t items)
{
    return (int)std::max<int64_t>(1, std::min<int64_t>(kTrackMaxBlocks, (items + kTrackThreads * 4 - 1) /
                                                                             (kTrackThreads * 4)));
}

template <int K>
__device__ __forceinline__ void block_sum(float (&v)[K], float (*sm)[kTrackThreads])
{
#pragma unroll
    for (int k = 0; k < K; ++k) sm[k][threadIdx.x] = v[k];
    __syncthreads();
    for (int w = kTrackThreads / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
#pragma unroll
            for (int k = 0; k < K; ++k) sm[k][threadIdx.x] += sm[k][threadIdx.x + w];
        }
        __syncthreads();
    }
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] = sm[k][0];
}

// ---- silhouette-masked colour + depth loss ----------------------------------

struct TrackImgs {
    int64_t hw;
    const float* C;   // [3][hw]
    const float* D;   // [hw]
    const float* A;   // [hw] silhouette
    const float* tC;  // [3][hw]
    const float* tD;  // [hw], 0 = no observation
    float thresh;
    int norm;  // 1 or 2
};

__device__ __forceinline__ float track_err(float e, int norm) { return norm == 2 ? e * e : fabsf(e); }
__device__ __forceinline__ float track_derr(float e, int norm)
{
    return norm == 2 ? 2.0f * e : (e > 0.0f ? 1.0f : (e < 0.0f ? -1.0f : 0.0f));
}

// per block: (masked colour error sum, masked depth error sum, observed-depth count)
__global__ void __launch_bounds__(kTrackThreads) k_track_partials(TrackImgs im, float* __restrict__ partial)
{
    __shared__ float sm[3][kTrackThreads];
    float v[3] = {0.0f, 0.0f, 0.0f};
    for (int64_t p = (int64_t)blockIdx.x * kTrackThreads + threadIdx.x; p < im.hw;
         p += (int64_t)gridDim.x * kTrackThreads) {
        const bool on = im.A[p] > im.thresh;
        const float td = im.tD[p];
        const bool obs = td > 0.0f;
        if (on) {
#pragma unroll
            for (int c = 0; c < 3; ++c) v[0] += track_err(im.C[c * im.hw + p] - im.tC[c * im.hw + p], im.norm);
            if (obs) v[1] += track_err(im.D[p] - td, im.norm);
        }
        if (obs) v[2] += 1.0f;
    }
    block_sum<3>(v, sm);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < 3; ++k) partial[3 * blockIdx.x + k] = v[k];
    }
}

// scal: [0] = 1/N, [1] = lam_d / |R| (0 without observations)
__global__ void __launch_bounds__(kTrackThreads) k_track_finish(const float* __restrict__ partial, int nb,
                                                                int64_t hw, float lam_d, float* __restrict__ loss,
                                                                float* __restrict__ scal)
{
    __shared__ double sm[3][kTrackThreads];
    double v[3] = {0.0, 0.0, 0.0};
    for (int i = threadIdx.x; i < nb; i += kTrackThreads)
        for (int k = 0; k < 3; ++k) v[k] += (double)partial[3 * i + k];
    for (int k = 0; k < 3; ++k) sm[k][threadIdx.x] = v[k];
    __syncthreads();
    for (int w = kTrackThreads / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            for (int k = 0; k < 3; ++k) sm[k][threadIdx.x] += sm[k][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double n_r = sm[2][0];
        const double lc = sm[0][0] / (double)hw;
        const double ld = n_r > 0.0 ? sm[1][0] / n_r : 0.0;
        if (loss) *loss = (float)(lc + (double)lam_d * ld);
        scal[0] = (float)(1.0 / (double)hw);
        scal[1] = n_r > 0.0 ? (float)((double)lam_d / n_r) : 0.0f;
    }
}

__global__ void __launch_bounds__(kTrackThreads) k_track_grad(TrackImgs im, const float* __restrict__ scal,
                                                              float* __restrict__ dlc, float* __restrict__ dld)
{
    const int64_t p = (int64_t)blockIdx.x * kTrackThreads + threadIdx.x;
    if (p >= im.hw) return;
    const bool on = im.A[p] > im.thresh;
    const float sc = scal[0], sd = scal[1];
#pragma unroll
    for (int c = 0; c < 3; ++c)
        dlc[c * im.hw + p] = on ? sc * track_derr(im.C[c * im.hw + p] - im.tC[c * im.hw + p], im.norm) : 0.0f;
    const float td = im.tD[p];
    dld[p] = (on && td > 0.0f) ? sd * track_derr(im.D[p] - td, im.norm) : 0.0f;
}

void launch_track_loss(int W, int H, const float* C, const float* D, const float* A, const float* tC,
                       const float* tD, float lam_d, int norm, float thresh, float* dlc, float* dld, float* loss,
                       float* partial, hipStream_t s)
{
    TrackImgs im{(int64_t)W * H, C, D, A, tC, tD, thresh, norm};
    const int nb = track_blocks(im.hw);
    float* scal = partial + 3 * nb;
    k_track_partials<<<nb, kTrackThreads, 0, s>>>(im, partial);
    k_track_finish<<<1, kTrackThreads, 0, s>>>(partial, nb, im.hw, lam_d, loss, scal);
    if (dlc && dld)
        k_track_grad<<<(unsigned)((im.hw + kTrackThreads - 1) / kTrackThreads), kTrackThreads, 0, s>>>(im, scal, dlc,
                                                                                                     dld);
}

int64_t track_partial_floats(int W, int H) { return 3 * (int64_t)track_blocks((int64_t)W * H) + 2; }

// ---- SSIM -------------------------------------------------------------------

constexpr int kSsimTile = 16;
constexpr int kSsimR = 5;  // 11-tap window
constexpr int kSsimHalo = kSsimTile + 2 * kSsimR;
constexpr float kSsimC1 = 0.01f * 0.01f;
constexpr float kSsimC2 = 0.03f * 0.03f;

struct SsimWin {
    float g[2 * kSsimR + 1];
};

// one 16 x 16 tile of one channel: window sums of x, y, x^2, y^2, x y; writes
// dS/d(mu_x) - 2 mu_x dS/d(s_xx) - mu_y dS/d(s_xy), dS/d(s_xx), dS/d(s_xy)
// (planes [3][3][H][W]) and the block's sum of S
__global__ void __launch_bounds__(256) k_ssim_fwd(int W, int H, const float* __restrict__ X,
                                                  const float* __restrict__ Y, SsimWin win, float* __restrict__ dm,
                                                  float* __restrict__ partial)
{
    __shared__ float sx[kSsimHalo][kSsimHalo + 1];
    __shared__ float sy[kSsimHalo][kSsimHalo + 1];
    __shared__ float hs[5][kSsimHalo][kSsimTile + 1];
    __shared__ float red[256];
    const int64_t hw = (int64_t)W * H;
    const int c = blockIdx.z;
    const float* x = X + c * hw;
    const float* y = Y + c * hw;
    const int u0 = blockIdx.x * kSsimTile - kSsimR, v0 = blockIdx.y * kSsimTile - kSsimR;
    for (int i = threadIdx.x; i < kSsimHalo * kSsimHalo; i += 256) {
        const int r = i / kSsimHalo, q = i - r * kSsimHalo;
        const int u = u0 + q, v = v0 + r;
        const bool in = u >= 0 && u < W && v >= 0 && v < H;
        sx[r][q] = in ? x[(int64_t)v * W + u] : 0.0f;
        sy[r][q] = in ? y[(int64_t)v * W + u] : 0.0f;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < kSsimHalo * kSsimTile; i += 256) {
        const int r = i / kSsimTile, q = i - r * kSsimTile;
        float a0 = 0.0f, a1 = 0.0f, a2 = 0.0f, a3 = 0.0f, a4 = 0.0f;
#pragma unroll
        for (int k = 0; k < 2 * kSsimR + 1; ++k) {
            const float g = win.g[k], xv = sx[r][q + k], yv = sy[r][q + k];
            a0 += g * xv;
            a1 += g * yv;
            a2 += g * xv * xv;
            a3 += g * yv * yv;
            a4 += g * xv * yv;
        }
        hs[0][r][q] = a0;
        hs[1][r][q] = a1;
        hs[2][r][q] = a2;
        hs[3][r][q] = a3;
        hs[4][r][q] = a4;
    }
    __syncthreads();
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
    float m[5] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int k = 0; k < 2 * kSsimR + 1; ++k) {
        const float g = win.g[k];
#pragma unroll
        for (int j = 0; j < 5; ++j) m[j] += g * hs[j][ty + k][tx];
    }
    const int u = blockIdx.x * kSsimTile + tx, v = blockIdx.y * kSsimTile + ty;
    float sval = 0.0f;
    if (u < W && v < H) {
        const float mx = m[0], my = m[1];
        const float sxx = m[2] - mx * mx, syy = m[3] - my * my, sxy = m[4] - mx * my;
        const float n1 = 2.0f * mx * my + kSsimC1, n2 = 2.0f * sxy + kSsimC2;
        const float d1 = mx * mx + my * my + kSsimC1, d2 = sxx + syy + kSsimC2;
        const float inv = 1.0f / (d1 * d2);
        const float sv = n1 * n2 * inv;
        const float ds_dmx = 2.0f * my * n2 * inv - sv * 2.0f * mx / d1;
        const float ds_dsxx = -sv / d2;
        const float ds_dsxy = 2.0f * n1 * inv;
        const int64_t p = (int64_t)v * W + u;
        dm[(0 * 3 + c) * hw + p] = ds_dmx - 2.0f * mx * ds_dsxx - my * ds_dsxy;
        dm[(1 * 3 + c) * hw + p] = ds_dsxx;
        dm[(2 * 3 + c) * hw + p] = ds_dsxy;
        sval = sv;
    }
    red[threadIdx.x] = sval;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        partial[((int64_t)blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x] = red[0];
}

// dL/dx = coef * (G * A + 2 x G * B + y G * Cm), added into dlc
__global__ void __launch_bounds__(256) k_ssim_bwd(int W, int H, const float* __restrict__ X,
                                                  const float* __restrict__ Y, SsimWin win,
                                                  const float* __restrict__ dm, float coef, float* __restrict__ dlc)
{
    __shared__ float sd[3][kSsimHalo][kSsimHalo + 1];
    __shared__ float hs[3][kSsimHalo][kSsimTile + 1];
    const int64_t hw = (int64_t)W * H;
    const int c = blockIdx.z;
    const int u0 = blockIdx.x * kSsimTile - kSsimR, v0 = blockIdx.y * kSsimTile - kSsimR;
    for (int i = threadIdx.x; i < kSsimHalo * kSsimHalo; i += 256) {
        const int r = i / kSsimHalo, q = i - r * kSsimHalo;
        const int u = u0 + q, v = v0 + r;
        const bool in = u >= 0 && u < W && v >= 0 && v < H;
        const int64_t p = (int64_t)v * W + u;
#pragma unroll
        for (int j = 0; j < 3; ++j) sd[j][r][q] = in ? dm[(j * 3 + c) * hw + p] : 0.0f;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < kSsimHalo * kSsimTile; i += 256) {
        const int r = i / kSsimTile, q = i - r * kSsimTile;
        float a[3] = {0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int k = 0; k < 2 * kSsimR + 1; ++k) {
            const float g = win.g[k];
#pragma unroll
            for (int j = 0; j < 3; ++j) a[j] += g * sd[j][r][q + k];
        }
#pragma unroll
        for (int j = 0; j < 3; ++j) hs[j][r][q] = a[j];
    }
    __syncthreads();
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
    const int u = blockIdx.x * kSsimTile + tx, v = blockIdx.y * kSsimTile + ty;
    if (u >= W || v >= H) return;
    float f[3] = {0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int k = 0; k < 2 * kSsimR + 1; ++k) {
        const float g = win.g[k];
#pragma unroll
        for (int j = 0; j < 3; ++j) f[j] += g * hs[j][ty + k][tx];
    }
    const int64_t p = (int64_t)v * W + u;
    const float xv = X[c * hw + p], yv = Y[c * hw + p];
    dlc[c * hw + p] += coef * (f[0] + 2.0f * xv * f[1] + yv * f[2]);
}

__global__ void __launch_bounds__(256) k_ssim_finish(const float* __restrict__ partial, int nb, double inv_m,
                                                     float weight, float* __restrict__ loss)
{
    __shared__ double sm[256];
    double a = 0.0;
    for (int i = threadIdx.x; i < nb; i += 256) a += (double)partial[i];
    sm[threadIdx.x] = a;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sm[threadIdx.x] += sm[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *loss = (float)((double)weight * (1.0 - sm[0] * inv_m));
}

int64_t ssim_partial_floats(int W, int H)
{
    return (int64_t)((W + kSsimTile - 1) / kSsimTile) * ((H + kSsimTile - 1) / kSsimTile) * 3;
}

void launch_ssim_loss(int W, int H, const float* X, const float* Y, float weight, float* dlc, float* loss, float* dm,
                      float* partial, hipStream_t s)
{
    SsimWin win;
    double g[2 * kSsimR + 1], sum = 0.0;
    for (int k = 0; k <= 2 * kSsimR; ++k) {
        const double d = k - kSsimR;
        g[k] = std::exp(-d * d / (2.0 * 1.5 * 1.5));
        sum += g[k];
    }
    for (int k = 0; k <= 2 * kSsimR; ++k) win.g[k] = (float)(g[k] / sum);
    const dim3 grid((W + kSsimTile - 1) / kSsimTile, (H + kSsimTile - 1) / kSsimTile, 3);
    const int nb = (int)(grid.x * grid.y * grid.z);
    const double m = 3.0 * (double)W * H;
    k_ssim_fwd<<<grid, 256, 0, s>>>(W, H, X, Y, win, dm, partial);
    if (loss) k_ssim_finish<<<1, 256, 0, s>>>(partial, nb, 1.0 / m, weight, loss);
    if (dlc) k_ssim_bwd<<<grid, 256, 0, s>>>(W, H, X, Y, win, dm, (float)(-(double)weight / m), dlc);
}

// ---- ICP ----------------------------------------------------------------------

constexpr int kIcpTile = 16;

// smallest and largest observed depth per 16 x 16 tile (+inf, -inf without observations)
__global__ void __launch_bounds__(256) k_icp_tile_range(const float* __restrict__ depth, int W, int H,
                                                        float2* __restrict__ trange)
{
    __shared__ float smin[256], smax[256];
    const int u = blockIdx.x * kIcpTile + (threadIdx.x & 15), v = blockIdx.y * kIcpTile + (threadIdx.x >> 4);
    float lo = __builtin_inff(), hi = -__builtin_inff();
    if (u < W && v < H) {
        const float z = depth[(int64_t)v * W + u];
        if (z > 0.0f) lo = hi = z;
    }
    smin[threadIdx.x] = lo;
    smax[threadIdx.x] = hi;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            smin[threadIdx.x] = fminf(smin[threadIdx.x], smin[threadIdx.x + w]);
            smax[threadIdx.x] = fmaxf(smax[threadIdx.x], smax[threadIdx.x + w]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) trange[blockIdx.y * gridDim.x + blockIdx.x] = make_float2(smin[0], smax[0]);
}

struct IcpArgs {
    int64_t n;
    const float* mean;  // [3][n]
    const float2* trange;  // [ceil(H/16)][ceil(W/16)] observed depth range per tile
    const float* depth; // [H][W] observed
    int W, H, stride;
    float fx, fy, cx, cy;
    float R[9], t[3];
    float tau;
    float weight;
    float* dmean;       // [3][n] added, or null
    float* partial;     // [grid][8]: loss, rho(3), phi(3), matched
};

constexpr int kIcpGroup = 16;  // lanes that search for one Gaussian

// 16 lanes per Gaussian: the tiles of its window are tested 16 at a time, and
// the stride-aligned pixels of each tile that passes are spread over the lanes.
// The nearest point is taken by (distance^2, pixel index), lowest first, so an
// exact tie goes to the first pixel in raster order whatever the visiting order.
__global__ void __launch_bounds__(kTrackThreads) k_icp(IcpArgs a)
{
    __shared__ float sm[8][kTrackThreads];
    float acc[8] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
    const float tau2 = a.tau * a.tau;
    const int s = a.stride;
    const int gl = threadIdx.x & (kIcpGroup - 1);
    const int gbase = (threadIdx.x & 63) & ~(kIcpGroup - 1);  // first lane of the group in its wave
    const int tx = (a.W + kIcpTile - 1) / kIcpTile;
    constexpr int GPB = kTrackThreads / kIcpGroup;
    for (int64_t i = (int64_t)blockIdx.x * GPB + threadIdx.x / kIcpGroup; i < a.n; i += (int64_t)gridDim.x * GPB) {
        const float mx = a.mean[i], my = a.mean[a.n + i], mz = a.mean[2 * a.n + i];
        const float x = fmaf(a.R[0], mx, fmaf(a.R[1], my, fmaf(a.R[2], mz, a.t[0])));
        const float y = fmaf(a.R[3], mx, fmaf(a.R[4], my, fmaf(a.R[5], mz, a.t[1])));
        const float z = fmaf(a.R[6], mx, fmaf(a.R[7], my, fmaf(a.R[8], mz, a.t[2])));
        if (!(z + a.tau > 0.0f)) continue;  // every observed point has depth > 0 (uniform in the group)
        int ulo = 0, uhi = a.W - 1, vlo = 0, vhi = a.H - 1;
        if (z > a.tau) {
            const float iz = 1.0f / z;
            const float ru = a.fx * a.tau * (1.0f + fabsf(x * iz)) / (z - a.tau) + 2.0f;
            const float rv = a.fy * a.tau * (1.0f + fabsf(y * iz)) / (z - a.tau) + 2.0f;
            const float uc = a.fx * x * iz + a.cx - 0.5f, vc = a.fy * y * iz + a.cy - 0.5f;
            ulo = (int)fmaxf(0.0f, floorf(uc - ru));
            uhi = (int)fminf((float)(a.W - 1), ceilf(uc + ru));
            vlo = (int)fmaxf(0.0f, floorf(vc - rv));
            vhi = (int)fminf((float)(a.H - 1), ceilf(vc + rv));
        }
        float best = __builtin_inff();
        int bpix = 0x7fffffff;
        if (ulo <= uhi && vlo <= vhi) {
            const int ti0 = ulo / kIcpTile, ti1 = uhi / kIcpTile, tj0 = vlo / kIcpTile, tj1 = vhi / kIcpTile;
            const int ntx = ti1 - ti0 + 1, ntile = ntx * (tj1 - tj0 + 1);
            for (int tb = 0; tb < ntile; tb += kIcpGroup) {
                const int t = tb + gl;
                bool pass = false;
                if (t < ntile) {
                    const float2 r = a.trange[(tj0 + t / ntx) * tx + ti0 + t % ntx];
                    pass = r.x < z + a.tau && r.y > z - a.tau;
                }
                uint32_t m = (uint32_t)(__ballot(pass) >> gbase) & 0xFFFFu;
                while (m) {
                    const int k = __builtin_ctz(m);
                    m &= m - 1u;
                    const int ti = ti0 + (tb + k) % ntx, tj = tj0 + (tb + k) / ntx;
                    const int u0 = (max(ulo, ti * kIcpTile) + s - 1) / s * s, u1 = min(uhi, ti * kIcpTile + kIcpTile - 1);
                    const int v0 = (max(vlo, tj * kIcpTile) + s - 1) / s * s, v1 = min(vhi, tj * kIcpTile + kIcpTile - 1);
                    if (u0 > u1 || v0 > v1) continue;
                    const int nu = (u1 - u0) / s + 1, np = nu * ((v1 - v0) / s + 1);
                    for (int idx = gl; idx < np; idx += kIcpGroup) {
                        const int u = u0 + (idx % nu) * s, v = v0 + (idx / nu) * s;
                        const int pix = v * a.W + u;
                        const float d = a.depth[pix];
                        if (!(d > 0.0f)) continue;
                        const float px = ((float)u + 0.5f - a.cx) / a.fx, py = ((float)v + 0.5f - a.cy) / a.fy;
                        const float ex = x - px * d, ey = y - py * d, ez = z - d;
                        const float d2 = ex * ex + ey * ey + ez * ez;
                        if (d2 < tau2 && (d2 < best || (d2 == best && pix < bpix))) {
                            best = d2;
                            bpix = pix;
                        }
                    }
                }
            }
        }
        // lexicographic minimum over the group's 16 lanes
#pragma unroll
        for (int off = kIcpGroup / 2; off > 0; off >>= 1) {
            const float ob = __shfl_xor(best, off, kIcpGroup);
            const int op = __shfl_xor(bpix, off, kIcpGroup);
            if (ob < best || (ob == best && op < bpix)) {
                best = ob;
                bpix = op;
            }
        }
        if (gl != 0 || !(best < tau2)) continue;
        const int u = bpix % a.W, v = bpix / a.W;
        const float d = a.depth[bpix];
        const float qx = ((float)u + 0.5f - a.cx) / a.fx * d, qy = ((float)v + 0.5f - a.cy) / a.fy * d, qz = d;
        const float ex = x - qx, ey = y - qy, ez = z - qz;
        const float gx = 2.0f * a.weight * ex, gy = 2.0f * a.weight * ey, gz = 2.0f * a.weight * ez;
        acc[0] += ex * ex + ey * ey + ez * ez;
        acc[1] += gx;
        acc[2] += gy;
        acc[3] += gz;
        acc[4] += y * gz - z * gy;
        acc[5] += z * gx - x * gz;
        acc[6] += x * gy - y * gx;
        acc[7] += 1.0f;
        if (a.dmean) {
            // R^T g
            a.dmean[i] += a.R[0] * gx + a.R[3] * gy + a.R[6] * gz;
            a.dmean[a.n + i] += a.R[1] * gx + a.R[4] * gy + a.R[7] * gz;
            a.dmean[2 * a.n + i] += a.R[2] * gx + a.R[5] * gy + a.R[8] * gz;
        }
    }
    block_sum<8>(acc, sm);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < 8; ++k) a.partial[8 * blockIdx.x + k] = acc[k];
    }
}

// loss (overwritten) = weight * sum; dpose (added) = (rho, phi); matched (overwritten)
__global__ void __launch_bounds__(256) k_icp_finish(const float* __restrict__ partial, int nb, float weight,
                                                    float* __restrict__ loss, float* __restrict__ dpose,
                                                    uint32_t* __restrict__ matched)
{
    __shared__ double sm[8][256];
    double v[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    for (int b = threadIdx.x; b < nb; b += 256)
#pragma unroll
        for (int k = 0; k < 8; ++k) v[k] += (double)partial[8 * b + k];
#pragma unroll
    for (int k = 0; k < 8; ++k) sm[k][threadIdx.x] = v[k];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
#pragma unroll
            for (int k = 0; k < 8; ++k) sm[k][threadIdx.x] += sm[k][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        if (loss) *loss = (float)((double)weight * sm[0][0]);
        if (dpose)
            for (int k = 0; k < 6; ++k) dpose[k] += (float)sm[1 + k][0];
        if (matched) *matched = (uint32_t)(sm[7][0] + 0.5);
    }
}

// one 16-lane group per Gaussian
int icp_blocks(int64_t n)
{
    constexpr int64_t GPB = kTrackThreads / kIcpGroup;
    return (int)std::max<int64_t>(1, std::min<int64_t>((n + GPB - 1) / GPB, 1 << 16));
}

int64_t icp_tile_floats(int W, int H)
{
    return 2 * (int64_t)((W + kIcpTile - 1) / kIcpTile) * ((H + kIcpTile - 1) / kIcpTile);
}

void launch_icp(int64_t n, const float* mean, const float* depth, int W, int H, float fx, float fy, float cx,
                float cy, const float R[9], const float t[3], float tau, int stride, float weight, float* dmean,
                float* loss, float* dpose, uint32_t* matched, float* partial, float* tmin, hipStream_t s)
{
    IcpArgs a;
    a.trange = reinterpret_cast<const float2*>(tmin);
    a.n = n;
    a.mean = mean;
    a.depth = depth;
    a.W = W;
    a.H = H;
    a.stride = stride;
    a.fx = fx;
    a.fy = fy;
    a.cx = cx;
    a.cy = cy;
    for (int k = 0; k < 9; ++k) a.R[k] = R[k];
    for (int k = 0; k < 3; ++k) a.t[k] = t[k];
    a.tau = tau;
    a.weight = weight;
    a.dmean = dmean;
    a.partial = partial;
    const int nb = icp_blocks(n);
    if (n > 0) {
        k_icp_tile_range<<<dim3((W + kIcpTile - 1) / kIcpTile, (H + kIcpTile - 1) / kIcpTile), 256, 0, s>>>(
            depth, W, H, reinterpret_cast<float2*>(tmin));
        k_icp<<<nb, kTrackThreads, 0, s>>>(a);
    }
    else launch_fill_f32(partial, 0.0f, 8, s);
    k_icp_finish<<<1, 256, 0, s>>>(partial, n > 0 ? nb : 1, weight, loss, dpose, matched);
}

}  // namespace vcgs
