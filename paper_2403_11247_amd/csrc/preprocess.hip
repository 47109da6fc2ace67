// Projection of 3D Gaussians to 2D splats (paper eqs. (2)-(3)) and its adjoint.
//
// Forward, one thread per Gaussian:
//   p = R mu + t; cull unless p.z > z_near and opacity >= 1/255;
//   Sigma = Rq S S^T Rq^T (Rq from the normalised quaternion), Sigma' = J W Sigma W^T J^T + 0.3 I,
//   conic = Sigma'^-1, (u, v) = (fx x/z + cx, fy y/z + cy),
//   radius r = ceil(sqrt(2 ln2 (e+1) lambda_max)), e = floor(log2(255 o)), which bounds every
//   pixel whose footprint o exp(-1/2 d^T conic d) reaches 1/255 (since ln(255 o) < (e+1) ln 2),
//   and the inclusive 16x16-tile rectangle of the pixels within r.
// The depth bits and the tile rectangle are integers decided by floating point, so they are
// computed in a fixed binary32 operation order with no contraction; a CPU program that follows
// the same order reproduces them bit for bit.
#include "internal.h"

namespace vcgs {

CamK make_camk(const vcgs_camera& c, uint32_t tile_base)
{
    CamK k;
    k.W = c.width; k.H = c.height;
    k.fx = c.fx; k.fy = c.fy; k.cx = c.cx; k.cy = c.cy; k.znear = c.z_near;
    k.tiles_x = (c.width + kTile - 1) / kTile;
    k.tiles_y = (c.height + kTile - 1) / kTile;
    // host float arithmetic, one rounding per operation (same order as the device code)
    volatile float hw = 0.5f * (float)c.width, hh = 0.5f * (float)c.height;
    volatile float qx = hw / c.fx, qy = hh / c.fy;
    k.limx = kClampFov * qx;
    k.limy = kClampFov * qy;
    k.tile_base = tile_base;
    return k;
}

PoseK make_posek(const vcgs_pose& p)
{
    PoseK k;
    for (int i = 0; i < 9; ++i) k.R[i] = p.R[i];
    for (int i = 0; i < 3; ++i) k.t[i] = p.t[i];
    return k;
}

struct KeyOut {
    bool vis;
    float X, Y, Z;
    float K[6];             // J W Rq S, so that Sigma' = K K^T
    float ca, cb, cc, det;  // Sigma' + 0.3 I entries and determinant
    float lam;              // its larger eigenvalue
    double ud, vd;          // screen position (binary64)
    float u, v;             // and rounded to binary32
    int tx0, ty0, tx1, ty1;
};

// The key path: binary32, evaluated left to right, no fused operations.
__device__ __forceinline__ KeyOut key_path(float x, float y, float z, float s0, float s1, float s2,
                                                     float qw, float qx, float qy, float qz, float o,
                                                     const CamK& cam, const PoseK& P)
{
#pragma clang fp contract(off)
    KeyOut r;
    r.vis = false;
    // camera point and screen position in binary64 (world coordinates of several
    // metres would otherwise cost ~1e-3 px), then rounded to binary32
    const double xd = x, yd = y, zd = z;
    const double Xd = (((double)P.R[0] * xd + (double)P.R[1] * yd) + (double)P.R[2] * zd) + (double)P.t[0];
    const double Yd = (((double)P.R[3] * xd + (double)P.R[4] * yd) + (double)P.R[5] * zd) + (double)P.t[1];
    const double Zd = (((double)P.R[6] * xd + (double)P.R[7] * yd) + (double)P.R[8] * zd) + (double)P.t[2];
    if (!(Zd > (double)cam.znear)) return r;
    if (!(o >= kAlphaMin)) return r;
    const double txd = Xd / Zd, tyd = Yd / Zd;
    r.ud = (double)cam.fx * txd + (double)cam.cx;
    r.vd = (double)cam.fy * tyd + (double)cam.cy;
    r.X = (float)Xd; r.Y = (float)Yd; r.Z = (float)Zd;
    r.u = (float)r.ud; r.v = (float)r.vd;
    const float txz = (float)txd, tyz = (float)tyd;
    const float n2 = ((qw * qw + qx * qx) + qy * qy) + qz * qz;
    if (n2 > 0.0f) {
        const float nr = __builtin_sqrtf(n2);
        qw = qw / nr; qx = qx / nr; qy = qy / nr; qz = qz / nr;
    } else {
        qw = 1.0f; qx = 0.0f; qy = 0.0f; qz = 0.0f;
    }
    const float xx = qx * qx, yy = qy * qy, zz = qz * qz;
    const float xy = qx * qy, xz = qx * qz, yz = qy * qz;
    const float wx = qw * qx, wy = qw * qy, wz = qw * qz;
    float q[9];
    q[0] = 1.0f - 2.0f * (yy + zz); q[1] = 2.0f * (xy - wz);        q[2] = 2.0f * (xz + wy);
    q[3] = 2.0f * (xy + wz);        q[4] = 1.0f - 2.0f * (xx + zz); q[5] = 2.0f * (yz - wx);
    q[6] = 2.0f * (xz - wy);        q[7] = 2.0f * (yz + wx);        q[8] = 1.0f - 2.0f * (xx + yy);
    float m[9];
#pragma unroll
    for (int i = 0; i < 3; ++i) { m[3 * i] = q[3 * i] * s0; m[3 * i + 1] = q[3 * i + 1] * s1; m[3 * i + 2] = q[3 * i + 2] * s2; }
    const float cxz = fminf(fmaxf(txz, -cam.limx), cam.limx);
    const float cyz = fminf(fmaxf(tyz, -cam.limy), cam.limy);
    const float j00 = cam.fx / r.Z, j02 = -(cam.fx * cxz) / r.Z;
    const float j11 = cam.fy / r.Z, j12 = -(cam.fy * cyz) / r.Z;
    float T[6];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        T[j] = j00 * P.R[j] + j02 * P.R[6 + j];
        T[3 + j] = j11 * P.R[3 + j] + j12 * P.R[6 + j];
    }
    // K = J W Rq S (2x3), Sigma' = K K^T
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int j = 0; j < 3; ++j)
            r.K[3 * a + j] = (T[3 * a] * m[j] + T[3 * a + 1] * m[3 + j]) + T[3 * a + 2] * m[6 + j];
    const float* K = r.K;
    const float s00 = (K[0] * K[0] + K[1] * K[1]) + K[2] * K[2];
    const float s01 = (K[0] * K[3] + K[1] * K[4]) + K[2] * K[5];
    const float s11 = (K[3] * K[3] + K[4] * K[4]) + K[5] * K[5];
    r.ca = s00 + kLowPass;
    r.cb = s01;
    r.cc = s11 + kLowPass;
    // det(Sigma' + 0.3 I) = det(K K^T) + 0.3 tr(K K^T) + 0.09, det(K K^T) by Cauchy-Binet: no cancellation
    const float m01 = K[0] * K[4] - K[1] * K[3];
    const float m02 = K[0] * K[5] - K[2] * K[3];
    const float m12 = K[1] * K[5] - K[2] * K[4];
    const float detk = (m01 * m01 + m02 * m02) + m12 * m12;
    r.det = (detk + kLowPass * (s00 + s11)) + kLowPass2;
    if (!(r.det > 0.0f)) return r;
    const float hd = 0.5f * (r.ca - r.cc);
    const float lam = 0.5f * (r.ca + r.cc) + __builtin_sqrtf(hd * hd + r.cb * r.cb);
    r.lam = lam;
    const float y255 = 255.0f * o;
    const int e = (int)((__float_as_uint(y255) >> 23) & 0xFFu) - 127;
    const float kf = kTwoLn2 * (float)(e + 1);
    const float rad = ceilf(__builtin_sqrtf(kf * lam));
    if (!(fabsf(r.u) < 1e30f) || !(fabsf(r.v) < 1e30f) || !(rad < 1e30f)) return r;
    float xlo = ceilf((r.u - rad) - 0.5f), xhi = floorf((r.u + rad) - 0.5f);
    float ylo = ceilf((r.v - rad) - 0.5f), yhi = floorf((r.v + rad) - 0.5f);
    xlo = fmaxf(xlo, 0.0f); xhi = fminf(xhi, (float)(cam.W - 1));
    ylo = fmaxf(ylo, 0.0f); yhi = fminf(yhi, (float)(cam.H - 1));
    if (xlo > xhi || ylo > yhi) return r;
    r.tx0 = (int)xlo / kTile; r.tx1 = (int)xhi / kTile;
    r.ty0 = (int)ylo / kTile; r.ty1 = (int)yhi / kTile;
    r.vis = true;
    return r;
}

// DEV: the table is read from device memory (tabp; a captured graph replays
// with the poses uploaded there), else from the kernel argument tab_val, which
// block 0 also copies to save (when set) for the launches of the backward.
template <bool DEV>
__global__ void __launch_bounds__(256) k_preprocess(ProjTab tab_val, const ProjTab* __restrict__ tabp,
                                                    ProjTab* __restrict__ save, const float* __restrict__ mean,
                                                    const float* __restrict__ scale, const float* __restrict__ quat,
                                                    const float* __restrict__ opac, const float* __restrict__ color,
                                                    Splat* __restrict__ rec, uint32_t* __restrict__ depth_key,
                                                    uint2* __restrict__ rect, uint32_t* __restrict__ count,
                                                    float* __restrict__ g2_zero, ZeroSegs z, int64_t ztotal)
{
    const ProjTab& tab = DEV ? *tabp : tab_val;
    const int64_t n = tab.n;
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    // the pass's counters, ranges and look-back words (read only by later launches)
    if (ztotal > 0) zero_segs(z, ztotal, e, (int64_t)gridDim.x * blockDim.x);
    if (!DEV && save && blockIdx.x == 0) {
        static_assert(sizeof(ProjTab) % 4 == 0, "table copied in words");
        const uint32_t* src = reinterpret_cast<const uint32_t*>(&tab_val);
        for (int i = threadIdx.x; i < (int)(sizeof(ProjTab) / 4); i += blockDim.x)
            reinterpret_cast<uint32_t*>(save)[i] = src[i];
    }
    if (e >= n * tab.n_views) return;
    const int v = (int)(e / n);
    const int64_t g = e - (int64_t)v * n;
    const CamK& cam = tab.cam[v];
    // the shared set, or view v's own set (views' SoA sets stored one after another)
    const int64_t vb = tab.per_view ? (int64_t)v * n : 0;  // view offset per attribute component
    const float* vm = mean + 3 * vb;
    const float* vs = scale + 3 * vb;
    const float* vq = quat + 4 * vb;
    const float o = opac[vb + g];
    const KeyOut k = key_path(vm[g], vm[n + g], vm[2 * n + g], vs[g], vs[n + g], vs[2 * n + g], vq[g], vq[n + g],
                              vq[2 * n + g], vq[3 * n + g], o, cam, tab.pose[v]);
    if (!k.vis) {
        depth_key[e] = 0xFFFFFFFFu;
        count[e] = 0u;
        rect[e] = make_uint2(0u, 0u);
        return;
    }
    // Eigen form of the inverse 2D covariance: d^T Sigma''^-1 d = p1^2 / lam + p2^2 / lmin with
    // p1 = d . e, p2 = d . e_perp, e the unit eigenvector of the larger eigenvalue lam; lmin = det / lam.
    // Both terms are non-negative, so evaluating it loses no precision for thin footprints.
    // The record holds the eigenvector scaled by s1 = sqrt(log2(e) / (2 lam)) and by
    // s2 = sqrt(log2(e) / (2 lmin)), so that the base-2 exponent of the footprint is
    // -(q1^2 + q2^2) with q1 = s1 p1 = d . (s1 e), q2 = s2 p2 = d . (s2 e_perp).
    const float lmin = k.det / k.lam;
    const float da = k.lam - k.ca, dc = k.lam - k.cc;
    float ex, ey;
    if (fabsf(da) >= fabsf(dc)) { ex = k.cb; ey = da; } else { ex = dc; ey = k.cb; }
    const float nrm = sqrtf(ex * ex + ey * ey);
    if (nrm > 0.0f) { ex /= nrm; ey /= nrm; } else { ex = 1.0f; ey = 0.0f; }
    const float s1 = sqrtf(kHalfLog2e / k.lam), s2 = sqrtf(kHalfLog2e / lmin);
    Splat sp;
    sp.a = make_float4(k.u, k.v, (float)(k.ud - (double)k.u), (float)(k.vd - (double)k.v));
    sp.b = make_float4(s1 * ex, s1 * ey, s2 * ex, s2 * ey);
    const float* vc = color + 3 * vb;
    sp.c = make_float4(o, vc[g], vc[n + g], vc[2 * n + g]);
    sp.d = make_float4(k.Z, s1, s2, 0.0f);
    rec[e] = sp;
    depth_key[e] = __float_as_uint(k.Z);
    count[e] = (uint32_t)((k.tx1 - k.tx0 + 1) * (k.ty1 - k.ty0 + 1));
    rect[e] = make_uint2((uint32_t)k.tx0 | ((uint32_t)k.ty0 << 16), (uint32_t)k.tx1 | ((uint32_t)k.ty1 << 16));
    if (g2_zero) {  // the backward's gradient slots of this entry start at zero
        float4* z = reinterpret_cast<float4*>(g2_zero + (int64_t)kG2 * e);
        z[0] = z[1] = z[2] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    }
}

void launch_preprocess(const ProjTab& t, ProjTab* t_dev, const vcgs_gaussians& g, Splat* rec,
                       uint32_t* depth_key, uint2* rect, uint32_t* count, float* g2_zero, hipStream_t s,
                       const ZeroSegs* zero, bool by_value)
{
    ZeroSegs z{};
    int64_t ztotal = 0;
    if (zero) {
        z = *zero;
        ztotal = zero_segs_normalise(z);
    }
    const int64_t total = t.n * t.n_views;
    if (total <= 0) {
        if (zero) launch_zero_u32(*zero, s);
        return;
    }
    const unsigned blocks = (unsigned)((total + 255) / 256);
    if (by_value)
        k_preprocess<false><<<blocks, 256, 0, s>>>(t, nullptr, t_dev, g.mean, g.scale, g.quat, g.opacity, g.color, rec,
                                                   depth_key, rect, count, g2_zero, z, ztotal);
    else
        k_preprocess<true><<<blocks, 256, 0, s>>>(t, t_dev, nullptr, g.mean, g.scale, g.quat, g.opacity, g.color, rec,
                                                  depth_key, rect, count, g2_zero, z, ztotal);
}

// ---------------------------------------------------------------------------
// Adjoint of the projection.  Recomputes the forward quantities in FP32 from
// the inputs and chains dL/d(u, v, conic, opacity, colour, depth) to the
// Gaussian attributes and to the pose tangent xi = (rho, phi) (left
// perturbation: d p = rho + phi x p, d Sigma_cam = phi^ Sigma_cam - Sigma_cam phi^).
// The pose 6-vector is reduced per block in a fixed order (deterministic).
// ---------------------------------------------------------------------------
constexpr int kBwdThreads = 256;

// Block barrier ordering LDS only (global stores may stay in flight).
__device__ __forceinline__ void pp_barrier()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

__global__ void __launch_bounds__(kBwdThreads) k_preprocess_bwd(
    const ProjTab* __restrict__ tabp, const float* __restrict__ mean, const float* __restrict__ scale,
    const float* __restrict__ quat, const uint32_t* __restrict__ count, const Splat* __restrict__ rec,
    const float* __restrict__ g2, float* __restrict__ d_mean, float* __restrict__ d_scale, float* __restrict__ d_quat,
    float* __restrict__ d_opac, float* __restrict__ d_color, float* __restrict__ pose_partial)
{
    __shared__ float red[kBwdThreads / 64][kMaxViews][6];  // per wave and view: its pose 6-vector total
    const ProjTab& tab = *tabp;
    const int64_t n = tab.n;
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    // gradients summed over the views in view order (shared set), or per view (own sets)
    float dmu[3] = {0, 0, 0}, dsc[3] = {0, 0, 0}, dqt[4] = {0, 0, 0, 0}, dop = 0.0f, dcol[3] = {0, 0, 0};
    for (int vw = 0; vw < tab.n_views; ++vw) {
    const CamK& cam = tab.cam[vw];
    const PoseK& P = tab.pose[vw];
    const int64_t e = (int64_t)vw * n + g;
    const int64_t vb = tab.per_view ? (int64_t)vw * n : 0;  // view offset per attribute component
    float pose6[6] = {0, 0, 0, 0, 0, 0};
    if (g < n) {
        const bool vis = count[e] != 0u;
        float gg[10];
        if (vis) {
            const float4 a = *reinterpret_cast<const float4*>(g2 + kG2 * e);
            const float4 b = *reinterpret_cast<const float4*>(g2 + kG2 * e + 4);
            const float4 c = *reinterpret_cast<const float4*>(g2 + kG2 * e + 8);
            // The compositing adjoint sums dL/dpower against the scaled pixel
            // offset in the footprint's eigen frame: a = (sum dP q1, sum dP q2,
            // sum dP q1^2, sum dP q1 q2), b.x = sum dP q2^2, with q1 = s1 p1,
            // q2 = s2 p2, p1 = d . e, p2 = d . e_perp, e = (ex, ey) and
            // s^2 = 1 / (2 ln2 lambda).  Since d = p1 e + p2 e_perp and power =
            // -1/2 d^T Q d with Q = i1 e e^T + i2 e_perp e_perp^T (i = 1 / lambda
            // = 2 ln2 s^2): dL/du = sum dP (Q d)_x, dL/dv = sum dP (Q d)_y, where
            // i1 p1 e = 2 ln2 q1 (s1 e); the conic terms -1/2 dx^2, -dx dy,
            // -1/2 dy^2 follow from the second moments of (p1, p2) rotated back.
            const float4 eb = rec[e].b;  // s1 ex, s1 ey, s2 ex, s2 ey
            const float4 ed = rec[e].d;  // depth, s1, s2
            const float r1 = 1.0f / ed.y, r2 = 1.0f / ed.z;
            const float ex = eb.x * r1, ey = eb.y * r1;
            gg[0] = 2.0f * kLn2 * (eb.x * a.x - eb.w * a.y);
            gg[1] = 2.0f * kLn2 * (eb.y * a.x + eb.z * a.y);
            const float m11 = a.z * (r1 * r1), m12 = a.w * (r1 * r2), m22 = b.x * (r2 * r2);
            const float exx = ex * ex, eyy = ey * ey, exy = ex * ey;
            gg[2] = -0.5f * ((exx * m11 - 2.0f * exy * m12) + eyy * m22);
            gg[3] = -(exy * (m11 - m22) + (exx - eyy) * m12);
            gg[4] = -0.5f * ((eyy * m11 + 2.0f * exy * m12) + exx * m22);
            gg[5] = b.y; gg[6] = b.z; gg[7] = b.w; gg[8] = c.x; gg[9] = c.y;
        } else {
#pragma unroll
            for (int i = 0; i < 10; ++i) gg[i] = 0.0f;
        }
        dop += gg[5];
        dcol[0] += gg[6]; dcol[1] += gg[7]; dcol[2] += gg[8];
        if (vis) {
            const float x = mean[3 * vb + g], y = mean[3 * vb + n + g], z = mean[3 * vb + 2 * n + g];
            const float X = P.R[0] * x + P.R[1] * y + P.R[2] * z + P.t[0];
            const float Y = P.R[3] * x + P.R[4] * y + P.R[5] * z + P.t[1];
            const float Z = P.R[6] * x + P.R[7] * y + P.R[8] * z + P.t[2];
            float qw = quat[4 * vb + g], qx = quat[4 * vb + n + g], qy = quat[4 * vb + 2 * n + g],
                  qz = quat[4 * vb + 3 * n + g];
            const float n2 = qw * qw + qx * qx + qy * qy + qz * qz;
            const bool qok = n2 > 0.0f;
            const float qn = qok ? sqrtf(n2) : 1.0f;
            if (qok) { const float iq = 1.0f / qn; qw *= iq; qx *= iq; qy *= iq; qz *= iq; }
            else { qw = 1.0f; qx = qy = qz = 0.0f; }
            const float s[3] = {scale[3 * vb + g], scale[3 * vb + n + g], scale[3 * vb + 2 * n + g]};
            float r[9];
            r[0] = 1.f - 2.f * (qy * qy + qz * qz); r[1] = 2.f * (qx * qy - qw * qz); r[2] = 2.f * (qx * qz + qw * qy);
            r[3] = 2.f * (qx * qy + qw * qz); r[4] = 1.f - 2.f * (qx * qx + qz * qz); r[5] = 2.f * (qy * qz - qw * qx);
            r[6] = 2.f * (qx * qz - qw * qy); r[7] = 2.f * (qy * qz + qw * qx); r[8] = 1.f - 2.f * (qx * qx + qy * qy);
            float M[9], S[9];
#pragma unroll
            for (int i = 0; i < 3; ++i)
#pragma unroll
                for (int j = 0; j < 3; ++j) M[3 * i + j] = r[3 * i + j] * s[j];
#pragma unroll
            for (int i = 0; i < 3; ++i)
#pragma unroll
                for (int j = 0; j < 3; ++j)
                    S[3 * i + j] = M[3 * i] * M[3 * j] + M[3 * i + 1] * M[3 * j + 1] + M[3 * i + 2] * M[3 * j + 2];
            const float iz = 1.0f / Z;
            const float txz = X * iz, tyz = Y * iz;
            const bool clx = txz < -cam.limx || txz > cam.limx;
            const bool cly = tyz < -cam.limy || tyz > cam.limy;
            const float cxz = fminf(fmaxf(txz, -cam.limx), cam.limx);
            const float cyz = fminf(fmaxf(tyz, -cam.limy), cam.limy);
            const float J[6] = {cam.fx * iz, 0.f, -cam.fx * cxz * iz, 0.f, cam.fy * iz, -cam.fy * cyz * iz};
            float T[6];
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int j = 0; j < 3; ++j) T[3 * a + j] = J[3 * a] * P.R[j] + J[3 * a + 1] * P.R[3 + j] + J[3 * a + 2] * P.R[6 + j];
            // Sigma' = K K^T with K = T M; determinant of Sigma' + 0.3 I without cancellation
            float Kf[6];
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int j = 0; j < 3; ++j) Kf[3 * a + j] = T[3 * a] * M[j] + T[3 * a + 1] * M[3 + j] + T[3 * a + 2] * M[6 + j];
            const float s00 = Kf[0] * Kf[0] + Kf[1] * Kf[1] + Kf[2] * Kf[2];
            const float s01 = Kf[0] * Kf[3] + Kf[1] * Kf[4] + Kf[2] * Kf[5];
            const float s11 = Kf[3] * Kf[3] + Kf[4] * Kf[4] + Kf[5] * Kf[5];
            const float Sp[3] = {s00 + kLowPass, s01, s11 + kLowPass};
            const float m01 = Kf[0] * Kf[4] - Kf[1] * Kf[3];
            const float m02 = Kf[0] * Kf[5] - Kf[2] * Kf[3];
            const float m12 = Kf[1] * Kf[5] - Kf[2] * Kf[4];
            const float det = (m01 * m01 + m02 * m02 + m12 * m12) + kLowPass * (s00 + s11) + kLowPass2;
            const float idet = 1.0f / det;
            const float Q[4] = {Sp[2] * idet, -Sp[1] * idet, -Sp[1] * idet, Sp[0] * idet};
            // conic gradient -> H = -Q G Q, G = [[gA, gB/2], [gB/2, gC]]
            const float Gm[4] = {gg[2], 0.5f * gg[3], 0.5f * gg[3], gg[4]};
            float QG[4], H[4];
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j) QG[2 * i + j] = Q[2 * i] * Gm[j] + Q[2 * i + 1] * Gm[2 + j];
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j) H[2 * i + j] = -(QG[2 * i] * Q[j] + QG[2 * i + 1] * Q[2 + j]);
            float HT[6], dT[6], dS[9];
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int j = 0; j < 3; ++j) HT[3 * a + j] = H[2 * a] * T[j] + H[2 * a + 1] * T[3 + j];
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int j = 0; j < 3; ++j)
                    dT[3 * a + j] = 2.0f * (HT[3 * a] * S[j] + HT[3 * a + 1] * S[3 + j] + HT[3 * a + 2] * S[6 + j]);
#pragma unroll
            for (int i = 0; i < 3; ++i)
#pragma unroll
                for (int j = 0; j < 3; ++j) dS[3 * i + j] = T[i] * HT[j] + T[3 + i] * HT[3 + j];
            float dJ[6];
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int k = 0; k < 3; ++k)
                    dJ[3 * a + k] = dT[3 * a] * P.R[3 * k] + dT[3 * a + 1] * P.R[3 * k + 1] + dT[3 * a + 2] * P.R[3 * k + 2];
            const float iz2 = iz * iz;
            float dpc[3];
            dpc[0] = gg[0] * cam.fx * iz;
            dpc[1] = gg[1] * cam.fy * iz;
            dpc[2] = -(gg[0] * cam.fx * X + gg[1] * cam.fy * Y) * iz2 + gg[9];
            dpc[2] += -(dJ[0] * cam.fx + dJ[4] * cam.fy) * iz2;
            dpc[2] += dJ[2] * cam.fx * cxz * iz2 + dJ[5] * cam.fy * cyz * iz2;
            if (!clx) {
                dpc[0] += -dJ[2] * cam.fx * iz2;
                dpc[2] += dJ[2] * cam.fx * X * iz2 * iz;
            }
            if (!cly) {
                dpc[1] += -dJ[5] * cam.fy * iz2;
                dpc[2] += dJ[5] * cam.fy * Y * iz2 * iz;
            }
#pragma unroll
            for (int i = 0; i < 3; ++i) dmu[i] += P.R[i] * dpc[0] + P.R[3 + i] * dpc[1] + P.R[6 + i] * dpc[2];
            // pose: camera-frame covariance Sc = W S W^T and its gradient Gc = J^T H J
            float WS[9], Sc[9], Gc[9];
#pragma unroll
            for (int i = 0; i < 3; ++i)
#pragma unroll
                for (int j = 0; j < 3; ++j) WS[3 * i + j] = P.R[3 * i] * S[j] + P.R[3 * i + 1] * S[3 + j] + P.R[3 * i + 2] * S[6 + j];
#pragma unroll
            for (int i = 0; i < 3; ++i)
#pragma unroll
                for (int j = 0; j < 3; ++j) {
                    Sc[3 * i + j] = WS[3 * i] * P.R[3 * j] + WS[3 * i + 1] * P.R[3 * j + 1] + WS[3 * i + 2] * P.R[3 * j + 2];
                    Gc[3 * i + j] = J[i] * (H[0] * J[j] + H[1] * J[3 + j]) + J[3 + i] * (H[2] * J[j] + H[3] * J[3 + j]);
                }
            // K = Sc Gc - Gc Sc ; only K01, K12, K20 are needed
            const float K01 = Sc[0] * Gc[1] + Sc[1] * Gc[4] + Sc[2] * Gc[7] - (Gc[0] * Sc[1] + Gc[1] * Sc[4] + Gc[2] * Sc[7]);
            const float K12 = Sc[3] * Gc[2] + Sc[4] * Gc[5] + Sc[5] * Gc[8] - (Gc[3] * Sc[2] + Gc[4] * Sc[5] + Gc[5] * Sc[8]);
            const float K20 = Sc[6] * Gc[0] + Sc[7] * Gc[3] + Sc[8] * Gc[6] - (Gc[6] * Sc[0] + Gc[7] * Sc[3] + Gc[8] * Sc[6]);
            pose6[0] = dpc[0]; pose6[1] = dpc[1]; pose6[2] = dpc[2];
            pose6[3] = (Y * dpc[2] - Z * dpc[1]) + 2.0f * K12;
            pose6[4] = (Z * dpc[0] - X * dpc[2]) + 2.0f * K20;
            pose6[5] = (X * dpc[1] - Y * dpc[0]) + 2.0f * K01;
            // Sigma = M M^T
            float dM[9];
#pragma unroll
            for (int i = 0; i < 3; ++i)
#pragma unroll
                for (int j = 0; j < 3; ++j)
                    dM[3 * i + j] = 2.0f * (dS[3 * i] * M[j] + dS[3 * i + 1] * M[3 + j] + dS[3 * i + 2] * M[6 + j]);
            float dr[9];
#pragma unroll
            for (int j = 0; j < 3; ++j) dsc[j] += dM[j] * r[j] + dM[3 + j] * r[3 + j] + dM[6 + j] * r[6 + j];
#pragma unroll
            for (int i = 0; i < 3; ++i)
#pragma unroll
                for (int j = 0; j < 3; ++j) dr[3 * i + j] = dM[3 * i + j] * s[j];
            float dq[4];
            dq[0] = 2.f * (-qz * dr[1] + qy * dr[2] + qz * dr[3] - qx * dr[5] - qy * dr[6] + qx * dr[7]);
            dq[1] = 2.f * (qy * dr[1] + qz * dr[2] + qy * dr[3] - 2.f * qx * dr[4] - qw * dr[5] + qz * dr[6] + qw * dr[7] - 2.f * qx * dr[8]);
            dq[2] = 2.f * (-2.f * qy * dr[0] + qx * dr[1] + qw * dr[2] + qx * dr[3] + qz * dr[5] - qw * dr[6] + qz * dr[7] - 2.f * qy * dr[8]);
            dq[3] = 2.f * (-2.f * qz * dr[0] - qw * dr[1] + qx * dr[2] + qw * dr[3] - 2.f * qz * dr[4] + qy * dr[5] + qx * dr[6] + qy * dr[7]);
            if (qok) {
                const float dot = qw * dq[0] + qx * dq[1] + qy * dq[2] + qz * dq[3];
                const float iq = 1.0f / qn;
                dqt[0] += (dq[0] - qw * dot) * iq;
                dqt[1] += (dq[1] - qx * dot) * iq;
                dqt[2] += (dq[2] - qy * dot) * iq;
                dqt[3] += (dq[3] - qz * dot) * iq;
            }
        }
    }
    // this view's pose 6-vector summed over the wave's lanes (a butterfly) and
    // parked per wave; the waves' totals are added after the view loop, so
    // the views need no block barrier
#pragma unroll
    for (int i = 0; i < 6; ++i) {
        float v = pose6[i];
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6][vw][i] = v;
    }
    // a view's own set takes its gradients here; a shared set after all views
    if (tab.per_view || vw == tab.n_views - 1) {
        if (g < n) {
            if (d_opac) d_opac[vb + g] = dop;
            if (d_color) {
                float* p = d_color + 3 * vb;
                p[g] = dcol[0]; p[n + g] = dcol[1]; p[2 * n + g] = dcol[2];
            }
            if (d_mean) {
                float* p = d_mean + 3 * vb;
                p[g] = dmu[0]; p[n + g] = dmu[1]; p[2 * n + g] = dmu[2];
            }
            if (d_scale) {
                float* p = d_scale + 3 * vb;
                p[g] = dsc[0]; p[n + g] = dsc[1]; p[2 * n + g] = dsc[2];
            }
            if (d_quat) {
                float* p = d_quat + 4 * vb;
                p[g] = dqt[0]; p[n + g] = dqt[1]; p[2 * n + g] = dqt[2]; p[3 * n + g] = dqt[3];
            }
        }
        dop = 0.0f;
#pragma unroll
        for (int i = 0; i < 3; ++i) dmu[i] = dsc[i] = dcol[i] = 0.0f;
#pragma unroll
        for (int i = 0; i < 4; ++i) dqt[i] = 0.0f;
    }
    }
    // per view, the four wave totals in wave order (deterministic)
    pp_barrier();
    for (int i = threadIdx.x; i < 6 * tab.n_views; i += kBwdThreads) {
        const int vw = i / 6, c = i - 6 * vw;
        pose_partial[((int64_t)vw * gridDim.x + blockIdx.x) * 6 + c] =
            ((red[0][vw][c] + red[1][vw][c]) + red[2][vw][c]) + red[3][vw][c];
    }
}

int preprocess_bwd_blocks(int64_t n) { return (int)((n + kBwdThreads - 1) / kBwdThreads); }

void launch_preprocess_bwd(const ProjTab& t, const ProjTab* t_dev, const vcgs_gaussians& g, const uint32_t* count,
                           const Splat* rec, const float* g2, const vcgs_gaussian_buffers& out, float* pose_partial,
                           int blocks, hipStream_t s)
{
    if (t.n <= 0) return;
    k_preprocess_bwd<<<blocks, kBwdThreads, 0, s>>>(t_dev, g.mean, g.scale, g.quat, count, rec, g2, out.mean,
                                                    out.scale, out.quat, out.opacity, out.color, pose_partial);
}

// Sum of the per-block pose partials in block order, one block per view (deterministic).
__global__ void __launch_bounds__(256) k_pose_reduce(const float* __restrict__ partial, int nblocks,
                                                     float* __restrict__ out)
{
    __shared__ double acc[4 * 6];
    const float* part = partial + (int64_t)blockIdx.x * nblocks * 6;
    double a[6] = {0, 0, 0, 0, 0, 0};
    for (int b = threadIdx.x; b < nblocks; b += 256)
#pragma unroll
        for (int i = 0; i < 6; ++i) a[i] += (double)part[6 * b + i];
    block_sum_f64<6>(a, acc);
    if (threadIdx.x == 0)
#pragma unroll
        for (int i = 0; i < 6; ++i) out[6 * blockIdx.x + i] = (float)a[i];
}

void launch_pose_reduce(const float* partial, int n_views, int nblocks, float* dl_dpose, hipStream_t s)
{
    if (n_views <= 0) return;
    k_pose_reduce<<<n_views, 256, 0, s>>>(partial, nblocks, dl_dpose);
}

}  // namespace vcgs
