/*
 * Oracle for the differentiable tile-based Gaussian rasterizer.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this file's library.  It shares no
 * code with the HIP path: it is written from the paper's equations and the
 * readings listed in the design notes, in plain C, with FP64 arithmetic for
 * every value that reaches an output, and FP32 only for the tile/depth keys
 * (the one place where floating point decides integers, taken in the
 * kernel's precision with the same operation order and no contraction).
 *
 * Build: gcc -O2 -ffp-contract=off -fno-fast-math -fopenmp -shared -fPIC.
 *
 * Paper passages followed (arXiv 2403.11247):
 *   eq. (1)  3D Gaussian  G(x) = o exp(-1/2 (x-mu)^T Sigma^-1 (x-mu))   [Sec. 3.1]
 *   eq. (2)  Sigma = R S S^T R^T                                        [Sec. 3.1]
 *   eq. (3)  Sigma' = J W Sigma W^T J^T                                 [Sec. 3.1]
 *   eqs. (16)-(18) front-to-back colour, depth and silhouette
 *            compositing  C = sum c_i f_i prod_{j<i} (1 - f_j)         [Sec. 3.5]
 *   pose: the camera is {R|t} with p_cam = R p_world + t                [Sec. 3]
 *   the renderer's backward to depth, pose and cumulative opacity       [Sec. 4, implementation details]
 *
 * Readings (the paper is silent on these):
 *   - pixel (i, j) is sampled at its centre (i + 0.5, j + 0.5);
 *   - footprint f_i(p) = min(0.99, o_i exp(P)),  P = -1/2 d^T Q d, Q = (Sigma' + 0.3 I)^-1,
 *     d = p - (u, v); a Gaussian whose f_i(p) < 1/255 is skipped at p;
 *   - front-to-back stop: the Gaussian that would bring the transmittance
 *     below 1e-4 is excluded and the pixel stops;
 *   - depth d_i = camera-space z of the mean; D is not normalised;
 *   - J clamps x/z and y/z to +-1.3 times the half-extent over the focal length;
 *   - a Gaussian is binned to every 16x16 tile that meets the pixel square
 *     of half-width r = ceil(sqrt(2 ln2 (e+1) lambda_max)), e = floor(log2(255 o)),
 *     which contains every pixel where f_i >= 1/255;
 *   - pose gradient: left perturbation T <- exp(xi^) T, xi = (rho, phi).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int32_t width, height;
    float fx, fy, cx, cy, z_near;
    int32_t tile;
} orc_camera;

/* thresholds of the footprint and the stop rule, as FP32 constants */
#define ORC_ALPHA_MIN (1.0f / 255.0f)
#define ORC_ALPHA_MAX (0.99f)
#define ORC_T_MIN (1e-4f)
#define ORC_LOWPASS (0.3f)
#define ORC_LOWPASS2 (0.09f)
#define ORC_CLAMP_FOV (1.3f)
#define ORC_TWO_LN2 (1.3862944f)

/* Bands in which an FP32 evaluation of the same footprint may fall on the
 * other side of a threshold.  The FP32 projection carries relative errors of
 * a few unit roundoffs (u = 2^-24) in the 2x3 factor of Sigma'; along the
 * minor axis of Sigma' + 0.3 I this becomes a relative error of about
 * 8 u cond in its smaller eigenvalue (cond = lambda_max / lambda_min), so the
 * exponent of the footprint is off by about 8 u cond |power|.  The band on
 * alpha is that bound plus a floor of 2e-5; the band on the stop
 * transmittance is 2e-4 plus the running sum, over the contributors, of each
 * alpha band times alpha / (1 - alpha). */
#define ORC_U32 (5.9604644775390625e-08)
#define ORC_BAND_ALPHA_FLOOR (2e-5)
#define ORC_BAND_T_FLOOR (2e-4)
/* With a decision form: the FP32 renderer evaluates the eigen form of the same
 * binary32 covariance; its exponent carries a few rounding errors, each
 * scaled at most by sqrt(cond) (a rounded pixel offset or eigenvector meets
 * the larger coefficient of a thin footprint), so its relative error is below
 * ORC_EVAL_ULPS u (1 + sqrt(cond)) (|power| + 1); the stop transmittance adds
 * two roundings per contributor. */
#define ORC_EVAL_ULPS (8.0)
#define ORC_BAND_T_FLOOR_DEC (0.0)

#define ORC_SPLAT 12

/* flag bits of an ambiguous pixel (a threshold decision lies within FP32 noise) */
#define ORC_FLAG_ALPHA 1u
#define ORC_FLAG_STOP 2u
#define ORC_FLAG_CLAMP 4u

static inline uint32_t f2u(float x) { uint32_t u; memcpy(&u, &x, 4); return u; }

/* ------------------------------------------------------------------------ */
/* Key path: depth bits and tile rectangle of every Gaussian.  The camera     */
/* point and screen position are binary64, everything after them binary32;  */
/* every operation is one IEEE operation, evaluated left to right.          */
/* ------------------------------------------------------------------------ */
/* The binary32 footprint covariance and tile rectangle of one Gaussian (the
 * key path).  Returns 0 when the Gaussian is culled. */
typedef struct {
    float Z, u, v;
    float ca, cb, cc, det, lam;   /* Sigma' + 0.3 I, its determinant and larger eigenvalue */
    int rect[4];
} orc_key32;

static int key32(int64_t n, int64_t g, const float* mean, const float* scale, const float* quat,
                 const float* opac, const orc_camera* cam, const float* Rc, const float* tc, orc_key32* out)
{
    const float limx = ORC_CLAMP_FOV * ((0.5f * (float)cam->width) / cam->fx);
    const float limy = ORC_CLAMP_FOV * ((0.5f * (float)cam->height) / cam->fy);
    /* camera point and screen position in binary64, then rounded to binary32 */
    const double xd = mean[g], yd = mean[n + g], zd = mean[2 * n + g];
    const double Xd = (((double)Rc[0] * xd + (double)Rc[1] * yd) + (double)Rc[2] * zd) + (double)tc[0];
    const double Yd = (((double)Rc[3] * xd + (double)Rc[4] * yd) + (double)Rc[5] * zd) + (double)tc[1];
    const double Zd = (((double)Rc[6] * xd + (double)Rc[7] * yd) + (double)Rc[8] * zd) + (double)tc[2];
    if (!(Zd > (double)cam->z_near)) return 0;
    const float o = opac[g];
    if (!(o >= ORC_ALPHA_MIN)) return 0;  /* never reaches 1/255 anywhere */
    const double txd = Xd / Zd, tyd = Yd / Zd;
    const double ud = (double)cam->fx * txd + (double)cam->cx;
    const double vd = (double)cam->fy * tyd + (double)cam->cy;
    const float Z = (float)Zd;
    const float txz = (float)txd, tyz = (float)tyd;
    const float u = (float)ud, v = (float)vd;
    /* rotation of the normalised quaternion, eq. (2) */
    float qw = quat[g], qx = quat[n + g], qy = quat[2 * n + g], qz = quat[3 * n + g];
    const float n2 = ((qw * qw + qx * qx) + qy * qy) + qz * qz;
    if (n2 > 0.0f) {
        const float nr = sqrtf(n2);
        qw = qw / nr; qx = qx / nr; qy = qy / nr; qz = qz / nr;
    } else {
        qw = 1.0f; qx = 0.0f; qy = 0.0f; qz = 0.0f;
    }
    const float xx = qx * qx, yy = qy * qy, zz = qz * qz;
    const float xy = qx * qy, xz = qx * qz, yz = qy * qz;
    const float wx = qw * qx, wy = qw * qy, wz = qw * qz;
    float r[9];
    r[0] = 1.0f - 2.0f * (yy + zz); r[1] = 2.0f * (xy - wz);        r[2] = 2.0f * (xz + wy);
    r[3] = 2.0f * (xy + wz);        r[4] = 1.0f - 2.0f * (xx + zz); r[5] = 2.0f * (yz - wx);
    r[6] = 2.0f * (xz - wy);        r[7] = 2.0f * (yz + wx);        r[8] = 1.0f - 2.0f * (xx + yy);
    const float s0 = scale[g], s1 = scale[n + g], s2 = scale[2 * n + g];
    float m[9];
    for (int i = 0; i < 3; ++i) { m[3 * i] = r[3 * i] * s0; m[3 * i + 1] = r[3 * i + 1] * s1; m[3 * i + 2] = r[3 * i + 2] * s2; }
    /* projection Jacobian with clamped x/z, y/z */
    const float cxz = fminf(fmaxf(txz, -limx), limx);
    const float cyz = fminf(fmaxf(tyz, -limy), limy);
    const float j00 = cam->fx / Z, j02 = -(cam->fx * cxz) / Z;
    const float j11 = cam->fy / Z, j12 = -(cam->fy * cyz) / Z;
    float T[6];
    for (int j = 0; j < 3; ++j) {
        T[j] = j00 * Rc[j] + j02 * Rc[6 + j];
        T[3 + j] = j11 * Rc[3 + j] + j12 * Rc[6 + j];
    }
    /* Sigma' = K K^T with K = J W R S (2x3), eqs. (2)-(3) */
    float K[6];
    for (int a = 0; a < 2; ++a)
        for (int j = 0; j < 3; ++j)
            K[3 * a + j] = (T[3 * a] * m[j] + T[3 * a + 1] * m[3 + j]) + T[3 * a + 2] * m[6 + j];
    const float s00 = (K[0] * K[0] + K[1] * K[1]) + K[2] * K[2];
    const float s01 = (K[0] * K[3] + K[1] * K[4]) + K[2] * K[5];
    const float s11 = (K[3] * K[3] + K[4] * K[4]) + K[5] * K[5];
    const float ca = s00 + ORC_LOWPASS;
    const float cb = s01;
    const float cc = s11 + ORC_LOWPASS;
    /* det(Sigma' + 0.3 I) = det(K K^T) + 0.3 tr(K K^T) + 0.09, det(K K^T) as the sum of squared 2x2 minors */
    const float m01 = K[0] * K[4] - K[1] * K[3];
    const float m02 = K[0] * K[5] - K[2] * K[3];
    const float m12 = K[1] * K[5] - K[2] * K[4];
    const float detk = (m01 * m01 + m02 * m02) + m12 * m12;
    const float det = (detk + ORC_LOWPASS * (s00 + s11)) + ORC_LOWPASS2;
    if (!(det > 0.0f)) return 0;
    const float hd = 0.5f * (ca - cc);
    const float lam = 0.5f * (ca + cc) + sqrtf(hd * hd + cb * cb);
    const float y255 = 255.0f * o;
    const int e = (int)((f2u(y255) >> 23) & 0xFFu) - 127;
    const float kf = ORC_TWO_LN2 * (float)(e + 1);
    const float rad = ceilf(sqrtf(kf * lam));
    if (!(fabsf(u) < 1e30f) || !(fabsf(v) < 1e30f) || !(rad < 1e30f)) return 0;
    float xlo = ceilf((u - rad) - 0.5f), xhi = floorf((u + rad) - 0.5f);
    float ylo = ceilf((v - rad) - 0.5f), yhi = floorf((v + rad) - 0.5f);
    xlo = fmaxf(xlo, 0.0f); xhi = fminf(xhi, (float)(cam->width - 1));
    ylo = fmaxf(ylo, 0.0f); yhi = fminf(yhi, (float)(cam->height - 1));
    if (xlo > xhi || ylo > yhi) return 0;
    const int tx0 = (int)xlo / cam->tile, tx1 = (int)xhi / cam->tile;
    const int ty0 = (int)ylo / cam->tile, ty1 = (int)yhi / cam->tile;
    out->Z = Z; out->u = u; out->v = v;
    out->ca = ca; out->cb = cb; out->cc = cc; out->det = det; out->lam = lam;
    out->rect[0] = tx0; out->rect[1] = ty0; out->rect[2] = tx1; out->rect[3] = ty1;
    return 1;
}

void orc_keys(int64_t n, const float* mean, const float* scale, const float* quat,
              const float* opac, const orc_camera* cam, const float* Rc, const float* tc,
              uint32_t* depth_bits, int32_t* rect, int32_t* count)
{
    for (int64_t g = 0; g < n; ++g) {
        orc_key32 k;
        depth_bits[g] = 0xFFFFFFFFu;
        rect[4 * g + 0] = rect[4 * g + 1] = rect[4 * g + 2] = rect[4 * g + 3] = 0;
        count[g] = 0;
        if (!key32(n, g, mean, scale, quat, opac, cam, Rc, tc, &k)) continue;
        for (int i = 0; i < 4; ++i) rect[4 * g + i] = k.rect[i];
        count[g] = (k.rect[2] - k.rect[0] + 1) * (k.rect[3] - k.rect[1] + 1);
        depth_bits[g] = f2u(k.Z);
    }
}

/* ------------------------------------------------------------------------ */
/* Pairs: one (key, gid) per (Gaussian, tile); key = tile << 32 | depth bits. */
/* Sorted ascending by key, equal keys by gid.                               */
/* ------------------------------------------------------------------------ */
typedef struct { uint64_t key; uint32_t gid; } orc_pair;

static int pair_cmp(const void* a, const void* b)
{
    const orc_pair* x = (const orc_pair*)a;
    const orc_pair* y = (const orc_pair*)b;
    if (x->key != y->key) return x->key < y->key ? -1 : 1;
    if (x->gid != y->gid) return x->gid < y->gid ? -1 : 1;
    return 0;
}

int64_t orc_pair_count(int64_t n, const int32_t* count)
{
    int64_t p = 0;
    for (int64_t g = 0; g < n; ++g) p += count[g];
    return p;
}

void orc_sort_pairs(int64_t n, const uint32_t* depth_bits, const int32_t* rect, const int32_t* count,
                    int32_t tiles_x, uint64_t* keys, uint32_t* gids)
{
    const int64_t P = orc_pair_count(n, count);
    orc_pair* pr = (orc_pair*)malloc(sizeof(orc_pair) * (size_t)(P > 0 ? P : 1));
    int64_t k = 0;
    for (int64_t g = 0; g < n; ++g) {
        if (count[g] == 0) continue;
        for (int ty = rect[4 * g + 1]; ty <= rect[4 * g + 3]; ++ty)
            for (int tx = rect[4 * g + 0]; tx <= rect[4 * g + 2]; ++tx) {
                pr[k].key = ((uint64_t)(uint32_t)(ty * tiles_x + tx) << 32) | depth_bits[g];
                pr[k].gid = (uint32_t)g;
                ++k;
            }
    }
    qsort(pr, (size_t)P, sizeof(orc_pair), pair_cmp);
    for (int64_t i = 0; i < P; ++i) { keys[i] = pr[i].key; gids[i] = pr[i].gid; }
    free(pr);
}

void orc_tile_ranges(int64_t P, const uint64_t* keys, int32_t n_tiles, uint32_t* ranges)
{
    for (int t = 0; t < n_tiles; ++t) { ranges[2 * t] = 0; ranges[2 * t + 1] = 0; }
    for (int64_t i = 0; i < P; ++i) {
        const uint32_t t = (uint32_t)(keys[i] >> 32);
        if (i == 0 || (uint32_t)(keys[i - 1] >> 32) != t) ranges[2 * t] = (uint32_t)i;
        if (i == P - 1 || (uint32_t)(keys[i + 1] >> 32) != t) ranges[2 * t + 1] = (uint32_t)(i + 1);
    }
}

/* ------------------------------------------------------------------------ */
/* FP64 projection, eqs. (2)-(3).                                            */
/* ------------------------------------------------------------------------ */
typedef struct {
    double pc[3];      /* camera point */
    double qh[4];      /* normalised quaternion */
    double qn;         /* |q| (0 for the degenerate case) */
    double r[9];       /* rotation of qh */
    double M[9];       /* r * diag(s) */
    double S[9];       /* 3D covariance */
    double xzc, yzc;   /* clamped x/z, y/z */
    int clx, cly;      /* clamp active */
    double J[6];       /* 2x3 Jacobian */
    double T[6];       /* J W */
    double a, b, c;    /* Sigma' + 0.3 I */
    double det;
    double conic[3];   /* A, B, C of the inverse */
    double u, v;
} orc_proj;

static void proj64(const double* mu, const double* s, const double* q, const orc_camera* cam,
                   const double* Rc, const double* tc, orc_proj* P)
{
    for (int i = 0; i < 3; ++i) P->pc[i] = Rc[3 * i] * mu[0] + Rc[3 * i + 1] * mu[1] + Rc[3 * i + 2] * mu[2] + tc[i];
    const double n2 = q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3];
    if (n2 > 0.0) {
        P->qn = sqrt(n2);
        for (int i = 0; i < 4; ++i) P->qh[i] = q[i] / P->qn;
    } else {
        P->qn = 0.0; P->qh[0] = 1.0; P->qh[1] = P->qh[2] = P->qh[3] = 0.0;
    }
    const double w = P->qh[0], x = P->qh[1], y = P->qh[2], z = P->qh[3];
    double* r = P->r;
    r[0] = 1 - 2 * (y * y + z * z); r[1] = 2 * (x * y - w * z);     r[2] = 2 * (x * z + w * y);
    r[3] = 2 * (x * y + w * z);     r[4] = 1 - 2 * (x * x + z * z); r[5] = 2 * (y * z - w * x);
    r[6] = 2 * (x * z - w * y);     r[7] = 2 * (y * z + w * x);     r[8] = 1 - 2 * (x * x + y * y);
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) P->M[3 * i + j] = r[3 * i + j] * s[j];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double acc = 0;
            for (int k = 0; k < 3; ++k) acc += P->M[3 * i + k] * P->M[3 * j + k];
            P->S[3 * i + j] = acc;
        }
    const double X = P->pc[0], Y = P->pc[1], Z = P->pc[2];
    const double limx = (double)ORC_CLAMP_FOV * (0.5 * cam->width / (double)cam->fx);
    const double limy = (double)ORC_CLAMP_FOV * (0.5 * cam->height / (double)cam->fy);
    const double txz = X / Z, tyz = Y / Z;
    P->clx = (txz < -limx || txz > limx);
    P->cly = (tyz < -limy || tyz > limy);
    P->xzc = txz < -limx ? -limx : (txz > limx ? limx : txz);
    P->yzc = tyz < -limy ? -limy : (tyz > limy ? limy : tyz);
    const double fx = cam->fx, fy = cam->fy;
    P->J[0] = fx / Z; P->J[1] = 0; P->J[2] = -fx * P->xzc / Z;
    P->J[3] = 0; P->J[4] = fy / Z; P->J[5] = -fy * P->yzc / Z;
    for (int a = 0; a < 2; ++a)
        for (int j = 0; j < 3; ++j) {
            double acc = 0;
            for (int k = 0; k < 3; ++k) acc += P->J[3 * a + k] * Rc[3 * k + j];
            P->T[3 * a + j] = acc;
        }
    double Sp[4];
    for (int a = 0; a < 2; ++a)
        for (int bb = 0; bb < 2; ++bb) {
            double acc = 0;
            for (int i = 0; i < 3; ++i)
                for (int j = 0; j < 3; ++j) acc += P->T[3 * a + i] * P->S[3 * i + j] * P->T[3 * bb + j];
            Sp[2 * a + bb] = acc;
        }
    P->a = Sp[0] + (double)ORC_LOWPASS;
    P->b = Sp[1];
    P->c = Sp[3] + (double)ORC_LOWPASS;
    P->det = P->a * P->c - P->b * P->b;
    P->conic[0] = P->c / P->det;
    P->conic[1] = -P->b / P->det;
    P->conic[2] = P->a / P->det;
    P->u = fx * txz + cam->cx;
    P->v = fy * tyz + cam->cy;
}

static void load_g(int64_t n, int64_t g, const double* mean, const double* scale, const double* quat,
                   double* mu, double* s, double* q)
{
    for (int i = 0; i < 3; ++i) { mu[i] = mean[i * n + g]; s[i] = scale[i * n + g]; }
    for (int i = 0; i < 4; ++i) q[i] = quat[i * n + g];
}

/* splat parameters of every Gaussian: (u, v, A, B, C, depth, cond, 0), where
 * cond = lambda_max / lambda_min of Sigma' + 0.3 I */
void orc_project(int64_t n, const double* mean, const double* scale, const double* quat,
                 const orc_camera* cam, const double* Rc, const double* tc, double* splat)
{
#pragma omp parallel for schedule(static)
    for (int64_t g = 0; g < n; ++g) {
        double mu[3], s[3], q[4];
        load_g(n, g, mean, scale, quat, mu, s, q);
        orc_proj P;
        proj64(mu, s, q, cam, Rc, tc, &P);
        double* o = splat + ORC_SPLAT * g;
        const double hd = 0.5 * (P.a - P.c), mid = 0.5 * (P.a + P.c);
        const double rt = sqrt(hd * hd + P.b * P.b);
        const double lmax = mid + rt, lmin = P.det / lmax;
        o[0] = P.u; o[1] = P.v; o[2] = P.conic[0]; o[3] = P.conic[1]; o[4] = P.conic[2]; o[5] = P.pc[2];
        o[6] = lmax / lmin;
        for (int i = 7; i < ORC_SPLAT; ++i) o[i] = 0.0;
    }
}

/* Decision form of every visible Gaussian: slots 7-11 of its splat record get
 * (1, ex, ey, 1/lambda_max, 1/lambda_min), the eigen form of the binary32
 * Sigma' + 0.3 I of the key path (its entries, determinant and larger
 * eigenvalue as the key path rounds them), evaluated exactly from there:
 * lambda_min = det / lambda_max, e the unit eigenvector of lambda_max.  Where
 * floating point decides an integer -- whether a Gaussian passes 1/255 at a
 * pixel, whether the pixel stops -- the decision is taken on this form, so it
 * sees the covariance the FP32 renderer sees; the values stay FP64. */
void orc_decision_form(int64_t n, const float* mean, const float* scale, const float* quat, const float* opac,
                       const orc_camera* cam, const float* Rc, const float* tc, double* splat)
{
#pragma omp parallel for schedule(static)
    for (int64_t g = 0; g < n; ++g) {
        double* o = splat + ORC_SPLAT * g;
        orc_key32 k;
        if (!key32(n, g, mean, scale, quat, opac, cam, Rc, tc, &k)) { for (int i = 7; i < ORC_SPLAT; ++i) o[i] = 0.0; continue; }
        const double lam = k.lam, lmin = (double)k.det / lam;
        const double da = lam - (double)k.ca, dc = lam - (double)k.cc;
        double ex, ey;
        if (fabs(da) >= fabs(dc)) { ex = k.cb; ey = da; } else { ex = dc; ey = k.cb; }
        const double nrm = sqrt(ex * ex + ey * ey);
        if (nrm > 0.0) { ex /= nrm; ey /= nrm; } else { ex = 1.0; ey = 0.0; }
        o[7] = 1.0; o[8] = ex; o[9] = ey; o[10] = 1.0 / lam; o[11] = 1.0 / lmin;
    }
}

/* ------------------------------------------------------------------------ */
/* Footprint and compositing, eqs. (1), (16)-(18).                           */
/* ------------------------------------------------------------------------ */
/* Value and decision of one footprint at one pixel.  The value (alpha, G,
 * power) is the FP64 footprint of eq. (1) on the image plane; the decisions
 * (skip below 1/255, clamp at 0.99, and the stop through alpha_dec) are taken
 * on the decision form when the record has one (slot 7), else on the value;
 * band bounds the relative error with which an FP32 renderer may evaluate
 * raw_dec. */
typedef struct { double G, raw, alpha, power, raw_dec, alpha_dec, band; int clamped; } orc_fp;

static inline orc_fp footprint(const double* sp, double o, double px, double py)
{
    orc_fp f;
    const double dx = px - sp[0], dy = py - sp[1];
    const double power = -0.5 * (sp[2] * dx * dx + sp[4] * dy * dy) - sp[3] * dx * dy;
    f.power = power;
    f.G = exp(power);
    f.raw = o * f.G;
    if (sp[7] != 0.0) {
        const double p1 = dx * sp[8] + dy * sp[9], p2 = dy * sp[8] - dx * sp[9];
        const double pd = -0.5 * (p1 * p1 * sp[10] + p2 * p2 * sp[11]);
        f.raw_dec = o * exp(pd);
        f.band = ORC_EVAL_ULPS * ORC_U32 * (1.0 + sqrt(sp[11] / sp[10])) * (fabs(pd) + 1.0);
    } else {
        f.raw_dec = f.raw;
        f.band = ORC_BAND_ALPHA_FLOOR + 8.0 * ORC_U32 * sp[6] * (fabs(power) + 1.0);
    }
    f.clamped = f.raw_dec > (double)ORC_ALPHA_MAX;
    f.alpha = f.clamped ? (double)ORC_ALPHA_MAX : f.raw;
    f.alpha_dec = f.clamped ? (double)ORC_ALPHA_MAX : f.raw_dec;
    return f;
}

static inline int near_rel(double x, double thr, double tol) { return fabs(x / thr - 1.0) < tol; }

/* Ambiguous decisions that a pixel's variants may take the other way; a pixel
 * with more keeps the FP64 decision beyond the first ORC_MAX_AMB. */
#define ORC_MAX_AMB 24

/* One contributor of a pixel, in front-to-back order. */
typedef struct { uint32_t g; double alpha, G, T; int clamped; } orc_contrib;

/* State of one front-to-back walk over a pixel's tile list. */
typedef struct {
    double T, c[3], d, a;
    int32_t last;     /* list entries up to and including the last contributor */
    uint8_t fl;       /* ambiguity flags met on the way */
    int n_amb;        /* ambiguous decisions met */
    uint64_t hash;    /* FNV-1a over the list positions of the contributors and the stop */
    size_t m;         /* contributors recorded */
} orc_walk;

/* Walks one pixel front to back, eqs. (16)-(18).  Every alpha-threshold and
 * stop decision is taken as in FP64, except that the i-th decision whose
 * margin lies within the FP32 band (an ambiguous one) is taken the other way
 * when choice[i] is 1 (i < nch).  Such a variant is what an FP32 evaluation of
 * the same footprints may legitimately produce.  When list is not NULL, the
 * contributors are recorded into *list (grown as needed). */
static void walk_px(const double* splat, const double* opac, const double* color, int64_t n,
                    const uint32_t* gids, uint32_t lo, uint32_t hi, double px, double py,
                    const uint8_t* choice, int nch, orc_walk* w, orc_contrib** list, size_t* cap)
{
    double T = 1.0, Td = 1.0, c0 = 0, c1 = 0, c2 = 0, d = 0, a = 0;
    double eT = 0.0;  /* running relative error bound of Td */
    int32_t last = 0;
    uint8_t fl = 0;
    int namb = 0;
    uint64_t h = 1469598103934665603ull;
    size_t m = 0;
    uint32_t k;
    for (k = lo; k < hi; ++k) {
        const uint32_t g = gids[k];
        const double* sp = splat + ORC_SPLAT * (size_t)g;
        const orc_fp f = footprint(sp, opac[g], px, py);
        int take = f.alpha_dec >= (double)ORC_ALPHA_MIN;
        if (near_rel(f.raw_dec, (double)ORC_ALPHA_MAX, f.band)) fl |= ORC_FLAG_CLAMP;
        if (near_rel(f.raw_dec, (double)ORC_ALPHA_MIN, f.band)) {
            fl |= ORC_FLAG_ALPHA;
            if (namb < nch && choice[namb]) take = !take;
            ++namb;
        }
        if (!take) continue;
        /* the transmittance the decision sees, and its error bound */
        const double Tdn = Td * (1.0 - f.alpha_dec);
        eT += f.band * f.alpha_dec / (1.0 - f.alpha_dec) + 2.0 * ORC_U32;
        int stop = Tdn < (double)ORC_T_MIN;
        if (near_rel(Tdn, (double)ORC_T_MIN, (sp[7] != 0.0 ? ORC_BAND_T_FLOOR_DEC : ORC_BAND_T_FLOOR) + eT)) {
            fl |= ORC_FLAG_STOP;
            if (namb < nch && choice[namb]) stop = !stop;
            ++namb;
        }
        if (stop) break;
        if (list) {
            if (m == *cap) {
                *cap = *cap ? 2 * *cap : 256;
                *list = (orc_contrib*)realloc(*list, *cap * sizeof(orc_contrib));
            }
            orc_contrib* e = *list + m;
            e->g = g; e->alpha = f.alpha; e->G = f.G; e->T = T; e->clamped = f.clamped;
        }
        ++m;
        const double wgt = f.alpha * T;
        c0 += wgt * color[g]; c1 += wgt * color[n + g]; c2 += wgt * color[2 * n + g];
        d += wgt * sp[5];
        a += wgt;
        T = T * (1.0 - f.alpha);
        Td = Tdn;
        last = (int32_t)(k - lo + 1);
        h = (h ^ (uint64_t)(k - lo)) * 1099511628211ull;
    }
    h = (h ^ (uint64_t)(k - lo) ^ 0x8000000000000000ull) * 1099511628211ull;
    w->T = T; w->c[0] = c0; w->c[1] = c1; w->c[2] = c2; w->d = d; w->a = a;
    w->last = last; w->fl = fl; w->n_amb = namb; w->hash = h; w->m = m;
}

/* Next choice vector in depth-first order (FP64 decisions first): flips the
 * last not yet flipped decision among the n_amb the previous walk met and
 * drops the ones after it.  Returns the new length, or -1 when every variant
 * has been visited. */
static int next_choice(uint8_t* choice, int nch, int n_amb)
{
    int len = n_amb < ORC_MAX_AMB ? n_amb : ORC_MAX_AMB;
    for (int i = nch; i < len; ++i) choice[i] = 0;
    for (int i = len - 1; i >= 0; --i)
        if (!choice[i]) { choice[i] = 1; return i + 1; }
    return -1;
}

/* Choice vector of variant v of a pixel (0 = every decision as in FP64).
 * Returns its length, or -1 when the pixel has no variant v. */
static int variant_choice(const double* splat, const double* opac, const double* color, int64_t n,
                          const uint32_t* gids, uint32_t lo, uint32_t hi, double px, double py, int v,
                          uint8_t* choice)
{
    int nch = 0;
    for (int i = 0; i < v; ++i) {
        orc_walk w;
        walk_px(splat, opac, color, n, gids, lo, hi, px, py, choice, nch, &w, NULL, NULL);
        nch = next_choice(choice, nch, w.n_amb);
        if (nch < 0) return -1;
    }
    return nch;
}

void orc_render_fwd(int64_t n, const double* splat, const double* opac, const double* color,
                    const orc_camera* cam, const double* bg, const uint32_t* ranges, const uint32_t* gids,
                    double* out_c, double* out_d, double* out_a, double* out_t, int32_t* out_n, uint8_t* out_f)
{
    const int W = cam->width, H = cam->height, tile = cam->tile;
    const int tiles_x = (W + tile - 1) / tile;
    const int64_t HW = (int64_t)W * H;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t p = 0; p < HW; ++p) {
        const int x = (int)(p % W), y = (int)(p / W);
        const int t = (y / tile) * tiles_x + (x / tile);
        orc_walk w;
        walk_px(splat, opac, color, n, gids, ranges[2 * t], ranges[2 * t + 1], x + 0.5, y + 0.5, NULL, 0, &w,
                NULL, NULL);
        out_c[p] = w.c[0] + w.T * bg[0]; out_c[HW + p] = w.c[1] + w.T * bg[1]; out_c[2 * HW + p] = w.c[2] + w.T * bg[2];
        out_d[p] = w.d; out_a[p] = w.a; out_t[p] = w.T; out_n[p] = w.last; out_f[p] = w.fl;
    }
}

/* Every outcome an FP32 renderer may legitimately produce at the listed
 * pixels: one per combination of the ambiguous decisions (the other side of an
 * alpha threshold or stop decision within FP32 noise), in depth-first order
 * with variant 0 the FP64 one.  out[i][v] = (C0, C1, C2, D, A, T_final,
 * n_contrib); nvar[i] = number of variants, or -1 when there are more than
 * maxv (only the first maxv are written). */
void orc_variants(int64_t n, const double* splat, const double* opac, const double* color,
                  const orc_camera* cam, const double* bg, const uint32_t* ranges, const uint32_t* gids,
                  int64_t npx, const int64_t* pix, int32_t maxv, double* out, int32_t* nvar)
{
    const int W = cam->width, tile = cam->tile;
    const int tiles_x = (W + tile - 1) / tile;
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t i = 0; i < npx; ++i) {
        const int64_t p = pix[i];
        const int x = (int)(p % W), y = (int)(p / W);
        const int t = (y / tile) * tiles_x + (x / tile);
        uint8_t choice[ORC_MAX_AMB];
        int nch = 0, v = 0;
        for (;;) {
            orc_walk w;
            walk_px(splat, opac, color, n, gids, ranges[2 * t], ranges[2 * t + 1], x + 0.5, y + 0.5, choice, nch,
                    &w, NULL, NULL);
            if (v == maxv) { v = -1; break; }
            double* o = out + ((size_t)i * maxv + v) * 7;
            o[0] = w.c[0] + w.T * bg[0]; o[1] = w.c[1] + w.T * bg[1]; o[2] = w.c[2] + w.T * bg[2];
            o[3] = w.d; o[4] = w.a; o[5] = w.T; o[6] = (double)w.last;
            ++v;
            nch = next_choice(choice, nch, w.n_amb);
            if (nch < 0) break;
        }
        nvar[i] = v;
    }
}

/* Per pixel, a hash of which list entries contribute and where the pixel
 * stops (FP64 decisions).  Two renders with the same tile lists and equal
 * hashes took every threshold decision the same way. */
void orc_decision_hash(int64_t n, const double* splat, const double* opac, const double* color,
                       const orc_camera* cam, const uint32_t* ranges, const uint32_t* gids, uint64_t* out)
{
    const int W = cam->width, H = cam->height, tile = cam->tile;
    const int tiles_x = (W + tile - 1) / tile;
    const int64_t HW = (int64_t)W * H;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t p = 0; p < HW; ++p) {
        const int x = (int)(p % W), y = (int)(p / W);
        const int t = (y / tile) * tiles_x + (x / tile);
        orc_walk w;
        walk_px(splat, opac, color, n, gids, ranges[2 * t], ranges[2 * t + 1], x + 0.5, y + 0.5, NULL, 0, &w,
                NULL, NULL);
        out[p] = w.hash;
    }
}

/* ------------------------------------------------------------------------ */
/* Hit counts (paper eq. (13), h): per Gaussian, the number of pixels whose   */
/* composite blends it (alpha >= 1/255, before the pixel stops).  amb counts, */
/* per Gaussian, the flagged pixels whose tile list holds it: there the FP32  */
/* renderer may take either side of a threshold, so its count may differ by  */
/* up to amb.                                                                 */
/* ------------------------------------------------------------------------ */
void orc_hit_counts(int64_t n, const double* splat, const double* opac, const orc_camera* cam,
                    const uint32_t* ranges, const uint32_t* gids, const uint8_t* flags, uint32_t* hits,
                    uint32_t* amb)
{
    const int W = cam->width, H = cam->height, tile = cam->tile;
    const int tiles_x = (W + tile - 1) / tile;
    const int64_t HW = (int64_t)W * H;
    memset(hits, 0, sizeof(uint32_t) * (size_t)n);
    memset(amb, 0, sizeof(uint32_t) * (size_t)n);
    size_t cap = 0;
    orc_contrib* list = NULL;
    for (int64_t p = 0; p < HW; ++p) {
        const int x = (int)(p % W), y = (int)(p / W);
        const int t = (y / tile) * tiles_x + (x / tile);
        orc_walk w;
        /* colours do not enter the hit count; the opacity array stands in for them */
        walk_px(splat, opac, opac, 0, gids, ranges[2 * t], ranges[2 * t + 1], x + 0.5, y + 0.5, NULL, 0, &w, &list,
                &cap);
        for (size_t i = 0; i < w.m; ++i) hits[list[i].g] += 1u;
        if (flags[p] & 3u)
            for (uint32_t k = ranges[2 * t]; k < ranges[2 * t + 1]; ++k) amb[gids[k]] += 1u;
    }
    free(list);
}

/* ------------------------------------------------------------------------ */
/* Adjoint of the compositing: exact derivative of the per-pixel sums.       */
/* g2 holds per Gaussian: du, dv, dA, dB, dC, dopacity, dr, dg, db, ddepth.  */
/* ------------------------------------------------------------------------ */
void orc_render_bwd_2d(int64_t n, const double* splat, const double* opac, const double* color,
                       const orc_camera* cam, const double* bg, const uint32_t* ranges, const uint32_t* gids,
                       const double* dl_dc, const double* dl_dd, const double* dl_da, const int32_t* variant,
                       double* g2)
{
    const int W = cam->width, H = cam->height, tile = cam->tile;
    const int tiles_x = (W + tile - 1) / tile;
    const int64_t HW = (int64_t)W * H;
    memset(g2, 0, sizeof(double) * 10 * (size_t)n);
    /* per-pixel contributor list */
    size_t cap = 0;
    orc_contrib* list = NULL;
    for (int64_t p = 0; p < HW; ++p) {
        const int x = (int)(p % W), y = (int)(p / W);
        const double px = x + 0.5, py = y + 0.5;
        const int t = (y / tile) * tiles_x + (x / tile);
        const double up[5] = {dl_dc[p], dl_dc[HW + p], dl_dc[2 * HW + p], dl_dd[p], dl_da[p]};
        /* forward, remembering every contributor; variant[p] > 0 selects which
         * side of the pixel's ambiguous decisions is taken (orc_variants order) */
        uint8_t choice[ORC_MAX_AMB];
        int nch = 0;
        if (variant && variant[p] > 0) {
            nch = variant_choice(splat, opac, color, n, gids, ranges[2 * t], ranges[2 * t + 1], px, py, variant[p],
                                 choice);
            if (nch < 0) continue;  /* no such variant: the pixel adds nothing */
        }
        orc_walk wk;
        walk_px(splat, opac, color, n, gids, ranges[2 * t], ranges[2 * t + 1], px, py, choice, nch, &wk, &list, &cap);
        const size_t m = wk.m;
        const double Tfin = wk.T;
        /* S holds sum_{j>i} x_j alpha_j T_j + T_final * bg_x for x = r, g, b, depth, 1 */
        double S[5] = {Tfin * bg[0], Tfin * bg[1], Tfin * bg[2], 0.0, 0.0};
        for (size_t ii = m; ii-- > 0;) {
            const uint32_t g = list[ii].g;
            const double a = list[ii].alpha, Tb = list[ii].T;
            const double xval[5] = {color[g], color[n + g], color[2 * n + g], splat[ORC_SPLAT * (size_t)g + 5], 1.0};
            /* d out_x / d alpha_i = x_i T_i - S_i / (1 - alpha_i) */
            double dl_dalpha = 0.0;
            for (int c = 0; c < 5; ++c) dl_dalpha += up[c] * (xval[c] * Tb - S[c] / (1.0 - a));
            double* gg = g2 + 10 * (size_t)g;
            const double w = a * Tb;
            gg[6] += w * up[0]; gg[7] += w * up[1]; gg[8] += w * up[2];
            gg[9] += w * up[3];
            if (!list[ii].clamped) {
                const double* sp = splat + ORC_SPLAT * (size_t)g;
                const double dx = px - sp[0], dy = py - sp[1];
                const double dl_dpow = dl_dalpha * a;  /* alpha = o exp(power) */
                gg[0] += dl_dpow * (sp[2] * dx + sp[3] * dy);
                gg[1] += dl_dpow * (sp[4] * dy + sp[3] * dx);
                gg[2] += dl_dpow * (-0.5 * dx * dx);
                gg[3] += dl_dpow * (-dx * dy);
                gg[4] += dl_dpow * (-0.5 * dy * dy);
                gg[5] += dl_dalpha * list[ii].G;
            }
            for (int c = 0; c < 5; ++c) S[c] += xval[c] * w;
        }
    }
    free(list);
}

/* ------------------------------------------------------------------------ */
/* Adjoint of the projection: 2D gradients -> mean, scale, quaternion,       */
/* opacity, colour, and the 6-vector pose gradient (rho, phi).               */
/* ------------------------------------------------------------------------ */
void orc_project_bwd(int64_t n, const double* mean, const double* scale, const double* quat,
                     const orc_camera* cam, const double* Rc, const double* tc, const int32_t* visible,
                     const double* g2, double* d_mean, double* d_scale, double* d_quat, double* d_opac,
                     double* d_color, double* d_pose)
{
    for (int i = 0; i < 6; ++i) d_pose[i] = 0.0;
    const double fx = cam->fx, fy = cam->fy;
    for (int64_t g = 0; g < n; ++g) {
        for (int i = 0; i < 3; ++i) { d_mean[i * n + g] = 0; d_scale[i * n + g] = 0; d_color[i * n + g] = 0; }
        for (int i = 0; i < 4; ++i) d_quat[i * n + g] = 0;
        d_opac[g] = 0;
        if (!visible[g]) continue;
        const double* gg = g2 + 10 * (size_t)g;
        d_opac[g] = gg[5];
        for (int i = 0; i < 3; ++i) d_color[i * n + g] = gg[6 + i];
        double mu[3], s[3], q[4];
        load_g(n, g, mean, scale, quat, mu, s, q);
        orc_proj P;
        proj64(mu, s, q, cam, Rc, tc, &P);
        const double X = P.pc[0], Y = P.pc[1], Z = P.pc[2];
        /* conic -> Sigma'' : H = -Q G Q, G = [[gA, gB/2], [gB/2, gC]] */
        const double Q[4] = {P.conic[0], P.conic[1], P.conic[1], P.conic[2]};
        const double Gm[4] = {gg[2], 0.5 * gg[3], 0.5 * gg[3], gg[4]};
        double QG[4], H[4];
        for (int i = 0; i < 2; ++i)
            for (int j = 0; j < 2; ++j) QG[2 * i + j] = Q[2 * i] * Gm[j] + Q[2 * i + 1] * Gm[2 + j];
        for (int i = 0; i < 2; ++i)
            for (int j = 0; j < 2; ++j) H[2 * i + j] = -(QG[2 * i] * Q[j] + QG[2 * i + 1] * Q[2 + j]);
        /* Sigma' = T Sigma T^T: dL/dT = 2 H T Sigma, dL/dSigma = T^T H T */
        double HT[6], dT[6], dS[9];
        for (int a = 0; a < 2; ++a)
            for (int j = 0; j < 3; ++j) HT[3 * a + j] = H[2 * a] * P.T[j] + H[2 * a + 1] * P.T[3 + j];
        for (int a = 0; a < 2; ++a)
            for (int j = 0; j < 3; ++j) {
                double acc = 0;
                for (int k = 0; k < 3; ++k) acc += HT[3 * a + k] * P.S[3 * k + j];
                dT[3 * a + j] = 2.0 * acc;
            }
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) dS[3 * i + j] = P.T[i] * HT[j] + P.T[3 + i] * HT[3 + j];
        /* T = J W: dL/dJ = dT W^T */
        double dJ[6];
        for (int a = 0; a < 2; ++a)
            for (int k = 0; k < 3; ++k) {
                double acc = 0;
                for (int j = 0; j < 3; ++j) acc += dT[3 * a + j] * Rc[3 * k + j];
                dJ[3 * a + k] = acc;
            }
        /* camera point gradient: projection (u, v), depth, and J's dependence */
        double dpc[3] = {0, 0, 0};
        dpc[0] += gg[0] * fx / Z;
        dpc[2] += -gg[0] * fx * X / (Z * Z);
        dpc[1] += gg[1] * fy / Z;
        dpc[2] += -gg[1] * fy * Y / (Z * Z);
        dpc[2] += gg[9];
        dpc[2] += dJ[0] * (-fx / (Z * Z)) + dJ[4] * (-fy / (Z * Z));
        /* J02 = -fx xzc / Z, xzc = X/Z unless clamped */
        dpc[2] += dJ[2] * (fx * P.xzc / (Z * Z));
        if (!P.clx) {
            dpc[0] += dJ[2] * (-fx / (Z * Z));
            dpc[2] += dJ[2] * (-fx / Z) * (-X / (Z * Z));
        }
        dpc[2] += dJ[5] * (fy * P.yzc / (Z * Z));
        if (!P.cly) {
            dpc[1] += dJ[5] * (-fy / (Z * Z));
            dpc[2] += dJ[5] * (-fy / Z) * (-Y / (Z * Z));
        }
        /* mean: p_c = W mu + t */
        for (int i = 0; i < 3; ++i) d_mean[i * n + g] = Rc[i] * dpc[0] + Rc[3 + i] * dpc[1] + Rc[6 + i] * dpc[2];
        /* pose: d p_c = rho + phi x p_c;  Sigma_c = W Sigma W^T gains phi^ Sigma_c - Sigma_c phi^ */
        double Sc[9], Gc[9], K[9];
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) {
                double acc = 0;
                for (int a = 0; a < 3; ++a)
                    for (int b = 0; b < 3; ++b) acc += Rc[3 * i + a] * P.S[3 * a + b] * Rc[3 * j + b];
                Sc[3 * i + j] = acc;
                Gc[3 * i + j] = P.J[i] * (H[0] * P.J[j] + H[1] * P.J[3 + j]) + P.J[3 + i] * (H[2] * P.J[j] + H[3] * P.J[3 + j]);
            }
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) {
                double acc = 0;
                for (int k = 0; k < 3; ++k) acc += Sc[3 * i + k] * Gc[3 * k + j] - Gc[3 * i + k] * Sc[3 * k + j];
                K[3 * i + j] = acc;
            }
        d_pose[0] += dpc[0]; d_pose[1] += dpc[1]; d_pose[2] += dpc[2];
        d_pose[3] += (Y * dpc[2] - Z * dpc[1]) + 2.0 * K[5];
        d_pose[4] += (Z * dpc[0] - X * dpc[2]) + 2.0 * K[6];
        d_pose[5] += (X * dpc[1] - Y * dpc[0]) + 2.0 * K[1];
        /* Sigma = M M^T: dL/dM = 2 dS M */
        double dM[9];
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) {
                double acc = 0;
                for (int k = 0; k < 3; ++k) acc += dS[3 * i + k] * P.M[3 * k + j];
                dM[3 * i + j] = 2.0 * acc;
            }
        double dr[9];
        for (int j = 0; j < 3; ++j) {
            double acc = 0;
            for (int i = 0; i < 3; ++i) acc += dM[3 * i + j] * P.r[3 * i + j];
            d_scale[j * n + g] = acc;
        }
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) dr[3 * i + j] = dM[3 * i + j] * s[j];
        /* rotation of a unit quaternion (w, x, y, z) */
        const double w = P.qh[0], x = P.qh[1], y = P.qh[2], z = P.qh[3];
        double dq[4];
        dq[0] = 2 * (-z * dr[1] + y * dr[2] + z * dr[3] - x * dr[5] - y * dr[6] + x * dr[7]);
        dq[1] = 2 * (y * dr[1] + z * dr[2] + y * dr[3] - 2 * x * dr[4] - w * dr[5] + z * dr[6] + w * dr[7] - 2 * x * dr[8]);
        dq[2] = 2 * (-2 * y * dr[0] + x * dr[1] + w * dr[2] + x * dr[3] + z * dr[5] - w * dr[6] + z * dr[7] - 2 * y * dr[8]);
        dq[3] = 2 * (-2 * z * dr[0] - w * dr[1] + x * dr[2] + w * dr[3] - 2 * z * dr[4] + y * dr[5] + x * dr[6] + y * dr[7]);
        if (P.qn > 0.0) {
            const double dot = w * dq[0] + x * dq[1] + y * dq[2] + z * dq[3];
            for (int i = 0; i < 4; ++i) d_quat[i * n + g] = (dq[i] - P.qh[i] * dot) / P.qn;
        }
    }
}
