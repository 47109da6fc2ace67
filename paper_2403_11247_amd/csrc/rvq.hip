// Residual vector quantization on the GPU (paper Sec. 3.4, eqs. (14)-(15)).
//
// Stage l assigns each vector x_n the code of C^l nearest to its residual
// r^l_n = x_n - xhat^{l-1}_n; xhat is the running sum of the picked codes.
// The loss of eq. (15) and its gradient to the codes (the residual sits under
// a stop-gradient) are accumulated in the same pass.
//
// The search is plain VALU work, one vector per lane, with the codes read as
// wave-uniform scalar operands: for each code the distance is D fused
// multiply-adds on a precomputed row (|c|^2, -2c), then a compare and two
// selects.  At the paper's sizes (P <= 256 codes, D <= 32) the compare and
// select are a sizeable part of the work and the whole search over a million
// vectors takes microseconds; matrix cores would also round the dot products in
// an order no CPU check can follow, while the pick is an integer that has to
// match one.  The 256 threads of a block hold the same 64 vectors and split the
// codebook in four contiguous quarters; after each stage the quarters' winners
// are merged through LDS in code order, which keeps the first index among
// equal distances.
//
// Decision arithmetic (binary32, no contraction beyond the explicit fmaf):
//   |c|^2 = c_0 c_0, then fmaf(c_j, c_j, .);  e = |c|^2, then fmaf(-2 c_j, r_j, .);
//   xhat_j += c_j and r_j = x_j - xhat_j.
// Code gradients: per-block sums of residuals and counts per code in LDS as
// 64-bit fixed point (2^-32 units; integer atomics are exact, so the sums do
// not depend on the order the lanes arrive in, and they run far faster than
// float atomics on LDS), blocks summed in binary64 in block order, then
// dL/dC = 2/(N P) (count * C - sum r).
#include "internal.h"

namespace vcgs {

constexpr int kRvqMaxGridPartial = 512;
constexpr int kRvqMaxGrid = 4096;

typedef __attribute__((address_space(4))) const float CFloat;

__host__ __device__ constexpr int rvq_row(int dm) { return dm + 4; }  // |c|^2, -2c (dm), padding

// fixed point of the code sums: 2^-32 units in two's complement (a block's sum
// of one residual component must stay below 2^31 in magnitude)
constexpr unsigned long long kRvqOne = 1ull << 32;
constexpr double kRvqUnit = 1.0 / 4294967296.0;
__device__ __forceinline__ unsigned long long rvq_fixed(float v)
{
    return (unsigned long long)__float2ll_rn(v * 4294967296.0f);  // scaling by 2^32 is exact
}

// per-code gradient row: D residual sums and the count, padded to an odd
// stride so that different codes fall in different LDS banks
__host__ __device__ constexpr int rvq_gstride(int d) { return (d + 1) | 1; }

int rvq_padded_dim(int d) { return d <= 4 ? 4 : d <= 8 ? 8 : d <= 16 ? 16 : 32; }

// one thread per (stage, code): row = (|c|^2, -2 c_0 .. -2 c_{D-1}, 0 ...)
__global__ void __launch_bounds__(256) k_rvq_table(int rows, int D, int dm, const float* __restrict__ books,
                                                   float* __restrict__ tab)
{
#pragma clang fp contract(off)
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= rows) return;
    const float* c = books + (int64_t)i * D;
    float* t = tab + (int64_t)i * rvq_row(dm);
    float s = c[0] * c[0];
    for (int j = 1; j < D; ++j) s = fmaf(c[j], c[j], s);
    t[0] = s;
    for (int j = 0; j < rvq_row(dm) - 1; ++j) t[1 + j] = j < D ? -2.0f * c[j] : 0.0f;
}

struct RvqArgs {
    int64_t n;
    int D, L, P;
    const float* tab;    // [L][P][row] in global memory (scalar-operand path)
    const float* books;  // [L][P][D]
    const float* x;      // [n][D]
    void* idx;           // [L][n], 1 or 4 bytes
    int idx_bytes;
    float* recon;        // [n][D] or null
    float* partial;      // [grid][pstride] or null: code sums and counts [L][P][rvq_gstride(D)], then the loss
    int grad;            // accumulate code sums
    int pstride;
};

// NT threads = NT / 256 vector groups of 64 at a time, each searched by four
// waves over the four quarters of the codebook.  LTAB: the rows (|c|^2, -2c)
// are built in LDS at the start and read as wave-uniform broadcasts; otherwise
// they are read from the global table as scalar operands.
template <int DM, bool LTAB, int NT>
__global__ void __launch_bounds__(NT) k_rvq_assign(RvqArgs a)
{
#pragma clang fp contract(off)
    constexpr int SLOTS = NT / 256;
    constexpr int S = rvq_row(DM);
    extern __shared__ float4 dyn4[];
    float* dyn = reinterpret_cast<float*>(dyn4);
    __shared__ float s_e[2][SLOTS][4][64];
    __shared__ int s_k[2][SLOTS][4][64];
    __shared__ float s_l[NT / 64];
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int slot = wv >> 2, w = wv & 3;
    const int k0 = (w * a.P) >> 2;
    const int k1 = ((w + 1) * a.P) >> 2;
    const int rows = a.L * a.P;
    float* s_tab = dyn;
    unsigned long long* s_grad = reinterpret_cast<unsigned long long*>(dyn + (LTAB ? rows * S : 0));
    const int E = a.grad ? rows * rvq_gstride(a.D) : 0;
    if (LTAB) {
        for (int r = threadIdx.x; r < rows; r += NT) {
            const float* c = a.books + (int64_t)r * a.D;
            float* t = s_tab + r * S;
            float sq = c[0] * c[0];
            for (int j = 1; j < a.D; ++j) sq = fmaf(c[j], c[j], sq);
            t[0] = sq;
            for (int j = 0; j < S - 1; ++j) t[1 + j] = j < a.D ? -2.0f * c[j] : 0.0f;
        }
    }
    for (int i = threadIdx.x; i < E; i += NT) s_grad[i] = 0ull;
    __syncthreads();
    float lsum = 0.0f;
    int phase = 0;
    const int64_t groups = (a.n + 63) >> 6;
    for (int64_t base = (int64_t)blockIdx.x * SLOTS; base < groups; base += (int64_t)gridDim.x * SLOTS) {
        const int64_t v = (base + slot) * 64 + lane;
        const bool valid = v < a.n;
        float xr[DM], xh[DM];
#pragma unroll
        for (int j = 0; j < DM; ++j) {
            xr[j] = (valid && j < a.D) ? a.x[v * a.D + j] : 0.0f;
            xh[j] = 0.0f;
        }
        for (int l = 0; l < a.L; ++l) {
            float r[DM];
#pragma unroll
            for (int j = 0; j < DM; ++j) r[j] = xr[j] - xh[j];
            float be = __builtin_inff();
            int bk = 0x7fffffff;
            if (LTAB) {
                const float4* t = reinterpret_cast<const float4*>(s_tab + (l * a.P + k0) * S);
#pragma unroll 2
                for (int k = k0; k < k1; ++k, t += S / 4) {
                    float row[S];
#pragma unroll
                    for (int q = 0; q < S / 4; ++q) {
                        const float4 f = t[q];
                        row[4 * q] = f.x;
                        row[4 * q + 1] = f.y;
                        row[4 * q + 2] = f.z;
                        row[4 * q + 3] = f.w;
                    }
                    float e = row[0];
#pragma unroll
                    for (int j = 0; j < DM; ++j) e = fmaf(row[1 + j], r[j], e);
                    if (e < be) {
                        be = e;
                        bk = k;
                    }
                }
            } else {
                // wave-uniform rows read through the constant address space: scalar loads
                const CFloat* t = (const CFloat*)(a.tab + ((int64_t)l * a.P + k0) * S);
#pragma unroll DM <= 8 ? 4 : 2
                for (int k = k0; k < k1; ++k, t += S) {
                    float e = t[0];
#pragma unroll
                    for (int j = 0; j < DM; ++j) e = fmaf(t[1 + j], r[j], e);
                    if (e < be) {
                        be = e;
                        bk = k;
                    }
                }
            }
            const int buf = phase & 1;
            ++phase;
            s_e[buf][slot][w][lane] = be;
            s_k[buf][slot][w][lane] = bk;
            __syncthreads();
            be = s_e[buf][slot][0][lane];
            bk = s_k[buf][slot][0][lane];
#pragma unroll
            for (int u = 1; u < 4; ++u) {
                const float e2 = s_e[buf][slot][u][lane];
                if (e2 < be) {
                    be = e2;
                    bk = s_k[buf][slot][u][lane];
                }
            }
            if (bk < 0 || bk >= a.P) bk = 0;  // non-finite distances everywhere
            if (valid && w == 0 && a.idx) {
                if (a.idx_bytes == 1)
                    static_cast<uint8_t*>(a.idx)[(int64_t)l * a.n + v] = (uint8_t)bk;
                else
                    static_cast<int32_t*>(a.idx)[(int64_t)l * a.n + v] = bk;
            }
            // the picked code, all of it before any accumulation (one wait, then the
            // atomics issue back to back); from LDS, -0.5 * (-2 c) is exact
            float cv[DM];
            if (LTAB) {
                const float4* row4 = reinterpret_cast<const float4*>(s_tab + (l * a.P + bk) * S);
                float row[S];
#pragma unroll
                for (int q4 = 0; q4 < S / 4; ++q4) {
                    const float4 f = row4[q4];
                    row[4 * q4] = f.x;
                    row[4 * q4 + 1] = f.y;
                    row[4 * q4 + 2] = f.z;
                    row[4 * q4 + 3] = f.w;
                }
#pragma unroll
                for (int j = 0; j < DM; ++j) cv[j] = -0.5f * row[1 + j];
            } else {
                const float* cg = a.books + ((int64_t)l * a.P + bk) * a.D;
#pragma unroll
                for (int j = 0; j < DM; ++j) cv[j] = j < a.D ? cg[j] : 0.0f;
            }
            unsigned long long* g = s_grad + (l * a.P + bk) * rvq_gstride(a.D);
            float q = 0.0f;
#pragma unroll
            for (int j = 0; j < DM; ++j) {
                if (j < a.D) {
                    const float d = r[j] - cv[j];
                    q = fmaf(d, d, q);
                    xh[j] = xh[j] + cv[j];
                }
            }
            if (valid && a.grad) {
#pragma unroll
                for (int j = 0; j < DM; ++j)
                    if (j < a.D && (j & 3) == w) atomicAdd(g + j, rvq_fixed(r[j]));
            }
            if (valid && a.partial && w == 0) {
                lsum += q;
                if (a.grad) atomicAdd(g + a.D, kRvqOne);
            }
        }
        if (valid && a.recon) {
#pragma unroll
            for (int j = 0; j < DM; ++j)
                if (j < a.D && (j & 3) == w) a.recon[v * a.D + j] = xh[j];
        }
    }
    if (a.partial) {
        if (w == 0) {
            for (int off = 32; off > 0; off >>= 1) lsum += __shfl_xor(lsum, off, 64);
        }
        if (lane == 0) s_l[wv] = lsum;
        __syncthreads();
        float* p = a.partial + (int64_t)blockIdx.x * a.pstride;
        for (int i = threadIdx.x; i < E; i += NT) p[i] = (float)((double)(long long)s_grad[i] * kRvqUnit);
        if (threadIdx.x == 0) {
            float t = 0.0f;
            for (int u = 0; u < SLOTS; ++u) t += s_l[4 * u];
            p[E] = t;
        }
    }
}

// Block partials summed in binary64 in a fixed order: grid.y takes the rows in
// runs of kRvqRun (4 slices of 8 rows, loads issued together); k_rvq_apply adds
// the runs in order.
constexpr int kRvqRun = 32;

__global__ void __launch_bounds__(256) k_rvq_reduce(const float* __restrict__ partial, int grid, int stride,
                                                    int entries, double* __restrict__ red)
{
    __shared__ double sm[4][64];
    const int lane = threadIdx.x & 63;
    const int s = threadIdx.x >> 6;
    const int e = blockIdx.x * 64 + lane;
    const int r0 = blockIdx.y * kRvqRun + s;
    float v[kRvqRun / 4];
#pragma unroll
    for (int i = 0; i < kRvqRun / 4; ++i) {
        const int r = r0 + 4 * i;
        v[i] = (e < entries && r < grid) ? partial[(int64_t)r * stride + e] : 0.0f;
    }
    double acc = 0.0;
#pragma unroll
    for (int i = 0; i < kRvqRun / 4; ++i) acc += (double)v[i];
    sm[s][lane] = acc;
    __syncthreads();
    if (s == 0 && e < entries)
        red[(int64_t)blockIdx.y * entries + e] = ((sm[0][lane] + sm[1][lane]) + sm[2][lane]) + sm[3][lane];
}

__device__ __forceinline__ double rvq_red(const double* red, int runs, int entries, int e)
{
    double a = 0.0;
    for (int y = 0; y < runs; ++y) a += red[(int64_t)y * entries + e];
    return a;
}

// dL/dC += 2/(N P) (count C - sum r); the loss = sum / (N P)
__global__ void __launch_bounds__(256) k_rvq_apply(int L, int P, int D, int grad, const float* __restrict__ books,
                                                   const double* __restrict__ red, int runs, double inv_np,
                                                   float* __restrict__ dbooks, float* __restrict__ loss)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    const int G = rvq_gstride(D);
    const int E = grad ? L * P * G : 0;
    if (i == 0 && loss) *loss = (float)(rvq_red(red, runs, E + 1, E) * inv_np);
    if (!grad || i >= L * P * D) return;
    const int row = i / D, j = i - row * D;
    const double cnt = rvq_red(red, runs, E + 1, row * G + D);
    const double sr = rvq_red(red, runs, E + 1, row * G + j);
    dbooks[i] += (float)(2.0 * inv_np * (cnt * (double)books[i] - sr));
}

constexpr int kRvqStaticLds = 16 * 1024 + 64;
constexpr int kRvqLdsLimit = 160 * 1024;

static int rvq_threads(int dm) { return dm <= 16 ? 1024 : 512; }

int rvq_grid(int64_t n, int D, bool partial)
{
    const int64_t slots = rvq_threads(rvq_padded_dim(D)) / 256;
    const int64_t blocks = ((n + 63) / 64 + slots - 1) / slots;
    return (int)std::max<int64_t>(1, std::min<int64_t>(blocks, partial ? kRvqMaxGridPartial : kRvqMaxGrid));
}

int64_t rvq_partial_floats(int64_t n, int L, int P, int D, bool grad)
{
    const int64_t stride = (grad ? (int64_t)L * P * rvq_gstride(D) : 0) + 1;
    return stride * rvq_grid(n, D, true);
}

int64_t rvq_red_doubles(int64_t n, int L, int P, int D, bool grad)
{
    const int64_t entries = (grad ? (int64_t)L * P * rvq_gstride(D) : 0) + 1;
    return entries * ((rvq_grid(n, D, true) + kRvqRun - 1) / kRvqRun);
}

// LDS beyond 64 KiB per block must be allowed per kernel; false if refused
template <int DM, bool LTAB>
static bool rvq_allow_lds()
{
    constexpr int NT = DM <= 16 ? 1024 : 512;
    static int state[64] = {};  // per device: 0 unknown, 1 allowed, -1 refused
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return false;
    if (state[dev] == 0)
        state[dev] = hipFuncSetAttribute((const void*)k_rvq_assign<DM, LTAB, NT>,
                                         hipFuncAttributeMaxDynamicSharedMemorySize,
                                         kRvqLdsLimit - kRvqStaticLds) == hipSuccess ? 1 : -1;
    return state[dev] > 0;
}

template <int DM>
static bool rvq_allow(bool ltab)
{
    return ltab ? rvq_allow_lds<DM, true>() : rvq_allow_lds<DM, false>();
}

template <int DM>
static void rvq_launch(bool ltab, int grid, size_t lds, const RvqArgs& a, hipStream_t s)
{
    constexpr int NT = DM <= 16 ? 1024 : 512;
    if (ltab)
        k_rvq_assign<DM, true, NT><<<grid, NT, lds, s>>>(a);
    else
        k_rvq_assign<DM, false, NT><<<grid, NT, lds, s>>>(a);
}

bool launch_rvq(int64_t n, int D, int L, int P, const float* books, const float* x, void* idx, int idx_bytes,
                float* recon, float* loss, float* dbooks, float* tab, float* partial, double* red, hipStream_t s)
{
    const bool want_partial = loss || dbooks;
    const int grad = dbooks ? 1 : 0;
    if (n <= 0) {
        if (loss) launch_fill_f32(loss, 0.0f, 1, s);
        return true;
    }
    const int dm = rvq_padded_dim(D);
    const int rows = L * P;
    const int E = grad ? rows * rvq_gstride(D) : 0;
    const size_t tab_bytes = (size_t)rows * rvq_row(dm) * sizeof(float);
    const size_t acc_bytes = (size_t)E * sizeof(unsigned long long);
    auto allow = [&](bool lt) {
        switch (dm) {
        case 4: return rvq_allow<4>(lt);
        case 8: return rvq_allow<8>(lt);
        case 16: return rvq_allow<16>(lt);
        default: return rvq_allow<32>(lt);
        }
    };
    const size_t lds_limit = (size_t)(kRvqLdsLimit - kRvqStaticLds);
    bool ltab = acc_bytes + tab_bytes <= lds_limit;
    if (ltab && acc_bytes + tab_bytes > 64 * 1024 - kRvqStaticLds) ltab = allow(true);
    if (!ltab && acc_bytes > 64 * 1024 - kRvqStaticLds && !allow(false)) {
        (void)hipGetLastError();
        return false;
    }
    (void)hipGetLastError();
    if (!ltab) k_rvq_table<<<(rows + 255) / 256, 256, 0, s>>>(rows, D, dm, books, tab);
    RvqArgs a;
    a.n = n;
    a.D = D;
    a.L = L;
    a.P = P;
    a.tab = tab;
    a.books = books;
    a.x = x;
    a.idx = idx;
    a.idx_bytes = idx_bytes;
    a.recon = recon;
    a.partial = want_partial ? partial : nullptr;
    a.grad = grad;
    a.pstride = E + 1;
    const int grid = rvq_grid(n, D, want_partial);
    const size_t lds = acc_bytes + (ltab ? tab_bytes : 0);
    switch (dm) {
    case 4: rvq_launch<4>(ltab, grid, lds, a, s); break;
    case 8: rvq_launch<8>(ltab, grid, lds, a, s); break;
    case 16: rvq_launch<16>(ltab, grid, lds, a, s); break;
    default: rvq_launch<32>(ltab, grid, lds, a, s); break;
    }
    if (!want_partial) return true;
    const int entries = E + 1;
    const int runs = (grid + kRvqRun - 1) / kRvqRun;
    k_rvq_reduce<<<dim3((entries + 63) / 64, runs), 256, 0, s>>>(partial, grid, a.pstride, entries, red);
    const int outs = std::max(1, grad ? L * P * D : 1);
    k_rvq_apply<<<(outs + 255) / 256, 256, 0, s>>>(L, P, D, grad, books, red, runs, 1.0 / ((double)n * P), dbooks,
                                                   loss);
    return true;
}

}  // namespace vcgs
