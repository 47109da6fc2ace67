// Stable LSD radix sort of (uint32 key, uint32 value) pairs and a device-wide
// exclusive scan, written for wave64.
//
// Radix pass (8-bit digit), reduce-then-scan:
//   1. histogram: per 4096-item block, digit counts (lanes with equal digits are
//      grouped by 8 ballots so one lane adds each group's count; no LDS atomics);
//      written digit-major, hist[d * nblocks + b];
//   2. exclusive scan of hist -> global offset of (digit d, block b);
//   3. scatter: each wave owns 1024 consecutive items of its block and ranks
//      them in order, 64 at a time, against its own per-digit counters, so
//      equal digits keep their input order (stable).
#include "internal.h"

namespace vcgs {

constexpr int kThreads = 256;
constexpr int kItems = 16;                      // per thread
constexpr int kBlockItems = kThreads * kItems;  // 4096
constexpr int kWaveItems = kBlockItems / 4;     // 1024 per wave
constexpr int kBins = 256;

__device__ __forceinline__ uint64_t lanemask_lt()
{
    const unsigned lane = __lane_id();
    return (lane == 0) ? 0ull : (~0ull >> (64 - lane));
}

// Mask of active lanes whose 8-bit digit equals this lane's.
__device__ __forceinline__ uint64_t match8(uint32_t d, uint64_t active)
{
    uint64_t m = active;
#pragma unroll
    for (int b = 0; b < 8; ++b) {
        const bool bit = (d >> b) & 1u;
        const uint64_t bal = __ballot(bit);
        m &= bit ? bal : ~bal;
    }
    return m;
}

int radix_blocks(int64_t n) { return (int)((n + kBlockItems - 1) / kBlockItems) > 0 ? (int)((n + kBlockItems - 1) / kBlockItems) : 1; }

__device__ __forceinline__ int64_t dev_count(int64_t cap, const uint32_t* dev)
{
    return dev ? min((int64_t)*dev, cap) : cap;
}

__global__ void __launch_bounds__(kThreads) k_radix_hist(const uint32_t* __restrict__ keys, int64_t cap,
                                                         const uint32_t* __restrict__ ndev, int shift,
                                                         uint32_t* __restrict__ hist, int nb)
{
    const int64_t n = dev_count(cap, ndev);
    __shared__ uint32_t h[4][kBins];
    const int w = threadIdx.x >> 6;
    for (int i = threadIdx.x; i < 4 * kBins; i += kThreads) (&h[0][0])[i] = 0u;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kBlockItems + (int64_t)w * kWaveItems;
#pragma unroll 4
    for (int r = 0; r < kWaveItems / 64; ++r) {
        const int64_t idx = base + r * 64 + __lane_id();
        const bool valid = idx < n;
        const uint32_t d = valid ? (keys[idx] >> shift) & 0xFFu : 0u;
        const uint64_t active = __ballot(valid);
        if (active == 0ull) break;
        const uint64_t m = match8(d, active);
        if (valid && (m & lanemask_lt()) == 0ull) h[w][d] += (uint32_t)__popcll(m);
    }
    __syncthreads();
    const uint32_t c = h[0][threadIdx.x] + h[1][threadIdx.x] + h[2][threadIdx.x] + h[3][threadIdx.x];
    hist[(int64_t)threadIdx.x * nb + blockIdx.x] = c;
}

__global__ void __launch_bounds__(kThreads) k_radix_scatter(const uint32_t* __restrict__ keys_in,
                                                            const uint32_t* __restrict__ vals_in,
                                                            uint32_t* __restrict__ keys_out,
                                                            uint32_t* __restrict__ vals_out, int64_t cap,
                                                            const uint32_t* __restrict__ ndev, int shift,
                                                            const uint32_t* __restrict__ offs, int nb)
{
    const int64_t n = dev_count(cap, ndev);
    __shared__ uint32_t cnt[4][kBins];
    const int w = threadIdx.x >> 6;
    const unsigned lane = __lane_id();
    for (int i = threadIdx.x; i < 4 * kBins; i += kThreads) (&cnt[0][0])[i] = 0u;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kBlockItems + (int64_t)w * kWaveItems;
    uint32_t key[kItems], val[kItems];
#pragma unroll
    for (int r = 0; r < kItems; ++r) {
        const int64_t idx = base + r * 64 + lane;
        key[r] = idx < n ? keys_in[idx] : 0u;
        val[r] = idx < n ? (vals_in ? vals_in[idx] : (uint32_t)idx) : 0u;
    }
    const uint64_t lt = lanemask_lt();
    // per-wave digit histogram
#pragma unroll
    for (int r = 0; r < kItems; ++r) {
        const bool valid = base + r * 64 + lane < n;
        const uint64_t active = __ballot(valid);
        if (active == 0ull) continue;
        const uint32_t d = (key[r] >> shift) & 0xFFu;
        const uint64_t m = match8(d, active);
        if (valid && (m & lt) == 0ull) cnt[w][d] += (uint32_t)__popcll(m);
    }
    __syncthreads();
    {
        const int d = threadIdx.x;
        uint32_t run = offs[(int64_t)d * nb + blockIdx.x];
#pragma unroll
        for (int ww = 0; ww < 4; ++ww) {
            const uint32_t c = cnt[ww][d];
            cnt[ww][d] = run;
            run += c;
        }
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kItems; ++r) {
        const bool valid = base + r * 64 + lane < n;
        const uint64_t active = __ballot(valid);
        if (active == 0ull) continue;
        const uint32_t d = (key[r] >> shift) & 0xFFu;
        const uint64_t m = match8(d, active);
        uint32_t pos = 0;
        if (valid) pos = cnt[w][d];
        const uint32_t rank = (uint32_t)__popcll(m & lt);
        if (valid && rank == 0u) cnt[w][d] = pos + (uint32_t)__popcll(m);
        if (valid) {
            keys_out[pos + rank] = key[r];
            vals_out[pos + rank] = val[r];
        }
    }
}

// ---------------------------------------------------------------------------
// Exclusive scan
// ---------------------------------------------------------------------------

__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v)
{
    const unsigned lane = __lane_id();
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t t = __shfl_up(v, o, 64);
        if (lane >= (unsigned)o) v += t;
    }
    return v;
}

// Exclusive scan of one value per thread over a 256-thread block; returns the
// exclusive prefix and writes the block total to *total.
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t v, uint32_t* total)
{
    __shared__ uint32_t ws[4];
    const int w = threadIdx.x >> 6;
    const uint32_t inc = wave_incl_scan(v);
    if (__lane_id() == 63) ws[w] = inc;
    __syncthreads();
    uint32_t off = 0, tot = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        if (i < w) off += ws[i];
        tot += ws[i];
    }
    __syncthreads();
    *total = tot;
    return off + inc - v;
}

__global__ void __launch_bounds__(kThreads) k_scan_reduce(const uint32_t* __restrict__ in, int64_t n,
                                                          uint32_t* __restrict__ sums)
{
    const int64_t base = (int64_t)blockIdx.x * kBlockItems;
    uint32_t s = 0;
#pragma unroll
    for (int i = 0; i < kItems; ++i) {
        const int64_t idx = base + i * kThreads + threadIdx.x;
        if (idx < n) s += in[idx];
    }
    uint32_t tot;
    (void)block_excl_scan(s, &tot);
    if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

// Block-local exclusive scan of a 4096-chunk plus an optional per-block base.
__global__ void __launch_bounds__(kThreads) k_scan_down(const uint32_t* __restrict__ in, uint32_t* __restrict__ out,
                                                        int64_t n, const uint32_t* __restrict__ bases,
                                                        uint32_t* __restrict__ total)
{
    const int64_t base = (int64_t)blockIdx.x * kBlockItems + (int64_t)threadIdx.x * kItems;
    uint32_t v[kItems];
    uint32_t s = 0;
#pragma unroll
    for (int i = 0; i < kItems; ++i) {
        const int64_t idx = base + i;
        v[i] = idx < n ? in[idx] : 0u;
        s += v[i];
    }
    uint32_t tot;
    uint32_t run = block_excl_scan(s, &tot) + (bases ? bases[blockIdx.x] : 0u);
#pragma unroll
    for (int i = 0; i < kItems; ++i) {
        const int64_t idx = base + i;
        if (idx < n) out[idx] = run;
        run += v[i];
    }
    if (total && threadIdx.x == kThreads - 1 && blockIdx.x == gridDim.x - 1) *total = run;
}

int64_t scan_temp_words(int64_t n)
{
    int64_t w = 0;
    while (n > kBlockItems) {
        n = (n + kBlockItems - 1) / kBlockItems;
        w += n;
    }
    return w + 1;
}

void exclusive_scan_u32(const uint32_t* in, uint32_t* out, int64_t n, uint32_t* total, uint32_t* tmp, hipStream_t s)
{
    if (n <= 0) {
        if (total) launch_fill_u32(total, 0u, 1, s);
        return;
    }
    const int64_t nb = (n + kBlockItems - 1) / kBlockItems;
    if (nb == 1) {
        k_scan_down<<<1, kThreads, 0, s>>>(in, out, n, nullptr, total);
        return;
    }
    uint32_t* sums = tmp;
    k_scan_reduce<<<(unsigned)nb, kThreads, 0, s>>>(in, n, sums);
    exclusive_scan_u32(sums, sums, nb, nullptr, tmp + nb, s);
    k_scan_down<<<(unsigned)nb, kThreads, 0, s>>>(in, out, n, sums, total);
}

int radix_sort_u32(uint32_t* keys, uint32_t* vals, bool identity_vals, Count n, int end_bit, const SortTemp& t,
                   hipStream_t s)
{
    if (n.cap <= 0) return 0;
    const int nb = radix_blocks(n.cap);
    uint32_t* kb[2] = {keys, t.keys_alt};
    uint32_t* vb[2] = {vals, t.vals_alt};
    int cur = 0;
    for (int shift = 0; shift < end_bit; shift += 8) {
        k_radix_hist<<<nb, kThreads, 0, s>>>(kb[cur], n.cap, n.dev, shift, t.hist, nb);
        exclusive_scan_u32(t.hist, t.hist, (int64_t)kBins * nb, nullptr, t.scan_tmp, s);
        k_radix_scatter<<<nb, kThreads, 0, s>>>(kb[cur], identity_vals ? nullptr : vb[cur], kb[cur ^ 1], vb[cur ^ 1],
                                                n.cap, n.dev, shift, t.hist, nb);
        identity_vals = false;
        cur ^= 1;
    }
    return cur;
}

}  // namespace vcgs
