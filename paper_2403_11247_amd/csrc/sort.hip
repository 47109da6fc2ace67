// Stable LSD radix sort of (uint32 key, uint32 value) pairs and a device-wide
// exclusive scan, written for wave64.
//
// Sort: one launch per 8-bit digit pass (single sweep), after one histogram
// launch for all passes:
//   1. histogram: every digit of every pass counted over the whole input;
//   2. per pass, each block takes the next partition (2048 or 4096 items; the partition
//      number comes from an atomic counter, so every lower partition is already
//      running), ranks its items stably (each wave walks its quarter of the
//      partition in order, 64 at a time, grouping equal digits with 8 ballots), publishes its
//      digit counts, and looks back over the published counts of the lower
//      partitions for its global offsets (decoupled look-back: a partition
//      publishes its own counts before it waits on anyone, so the wait always
//      ends; eight predecessors are read at a time); items are then staged in LDS in digit order and written out so
//      that consecutive threads write consecutive addresses of a digit's run.
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

// Items per thread of a sort pass: small sorts (e.g. the depth sort over the
// Gaussians) use 2048-item partitions, so that more partitions run at once;
// large ones (the tile sort over the pairs) 4096.
constexpr int64_t kSmallSort = 1 << 20;
int sort_items(int64_t cap) { return cap <= kSmallSort ? 8 : 16; }
static int radix_blocks_items(int64_t cap, int items)
{
    const int64_t part = (int64_t)kThreads * items;
    return (int)std::max<int64_t>(1, (cap + part - 1) / part);
}
int radix_blocks(int64_t cap) { return radix_blocks_items(cap, sort_items(cap)); }

__device__ __forceinline__ int64_t dev_count(int64_t cap, const uint32_t* dev)
{
    return dev ? min((int64_t)*dev, cap) : cap;
}

// ---------------------------------------------------------------------------
// Exclusive scan
// ---------------------------------------------------------------------------

// Sums in the scan saturate at kScanSat: a pair count of 2^31 or more reads as
// 2^31 instead of wrapping, so the callers' limit of 2^30 - 1 pairs refuses it.
// min(a + b, kScanSat) is associative, so every prefix below the bound is exact.
constexpr uint32_t kScanSat = 0x80000000u;
__device__ __forceinline__ uint32_t sat_add(uint32_t a, uint32_t b)
{
    const uint32_t s = a + b;
    return (s < a || s > kScanSat) ? kScanSat : s;
}

__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v)
{
    const unsigned lane = __lane_id();
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t t = __shfl_up(v, o, 64);
        if (lane >= (unsigned)o) v = sat_add(v, t);
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
    const uint32_t prev = __shfl_up(inc, 1, 64);
    __syncthreads();
    uint32_t off = 0, tot = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        if (i < w) off = sat_add(off, ws[i]);
        tot = sat_add(tot, ws[i]);
    }
    __syncthreads();
    *total = tot;
    return sat_add(off, __lane_id() == 0 ? 0u : prev);
}

__global__ void __launch_bounds__(kThreads) k_scan_reduce(const uint32_t* __restrict__ in, int64_t n,
                                                          uint32_t* __restrict__ sums)
{
    const int64_t base = (int64_t)blockIdx.x * kBlockItems;
    uint32_t s = 0;
#pragma unroll
    for (int i = 0; i < kItems; ++i) {
        const int64_t idx = base + i * kThreads + threadIdx.x;
        if (idx < n) s = sat_add(s, in[idx]);
    }
    uint32_t tot;
    (void)block_excl_scan(s, &tot);
    if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

// Block-local exclusive scan of a 4096-chunk plus an optional per-block base.
// Loads and stores are coalesced (consecutive threads, consecutive words) and
// transposed through LDS, so that each thread scans 16 consecutive items.
__device__ __forceinline__ int scan_pad(int i) { return i + (i >> 4); }  // one spare word per 16: no bank conflicts

__global__ void __launch_bounds__(kThreads) k_scan_down(const uint32_t* __restrict__ in, uint32_t* __restrict__ out,
                                                        int64_t n, const uint32_t* __restrict__ bases,
                                                        uint32_t* __restrict__ total)
{
    __shared__ uint32_t tile[kBlockItems + kBlockItems / 16];
    const int64_t base = (int64_t)blockIdx.x * kBlockItems;
#pragma unroll
    for (int i = 0; i < kItems; ++i) {
        const int k = i * kThreads + threadIdx.x;
        tile[scan_pad(k)] = base + k < n ? in[base + k] : 0u;
    }
    __syncthreads();
    uint32_t v[kItems];
    uint32_t s = 0;
#pragma unroll
    for (int i = 0; i < kItems; ++i) {
        v[i] = tile[scan_pad(threadIdx.x * kItems + i)];
        s = sat_add(s, v[i]);
    }
    uint32_t tot;
    uint32_t run = sat_add(block_excl_scan(s, &tot), bases ? bases[blockIdx.x] : 0u);
#pragma unroll
    for (int i = 0; i < kItems; ++i) {
        tile[scan_pad(threadIdx.x * kItems + i)] = run;
        run = sat_add(run, v[i]);
    }
    if (total && threadIdx.x == kThreads - 1 && blockIdx.x == gridDim.x - 1) *total = run;
    __syncthreads();
#pragma unroll
    for (int i = 0; i < kItems; ++i) {
        const int k = i * kThreads + threadIdx.x;
        if (base + k < n) out[base + k] = tile[scan_pad(k)];
    }
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

// ---------------------------------------------------------------------------
// Pair offsets: gathered tile counts and their exclusive scan in one pass
// ---------------------------------------------------------------------------

// Look-back words, one per 4096-entry partition: the partition's own sum
// (flag kPsAgg) or the sum of it and every lower partition (kPsInc) in the
// low 32 bits.  Word 0 is the partition counter.
constexpr unsigned long long kPsAgg = 1ull << 62, kPsInc = 2ull << 62, kPsFlags = 3ull << 62;

int64_t pair_scan_words(int64_t n) { return 2 * ((std::max<int64_t>(n, 0) + kBlockItems - 1) / kBlockItems + 1); }

__device__ __forceinline__ unsigned long long load_agent64(const unsigned long long* p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void store_agent64(unsigned long long* p, unsigned long long v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Saturating sum over the 64 lanes, result in every lane.
__device__ __forceinline__ uint32_t wave_sum_sat(uint32_t v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = sat_add(v, (uint32_t)__shfl_xor((int)v, o, 64));
    return v;
}

// cnt[k] = count[order[k]] for k below the device count (0 up to n_all),
// offs = the exclusive prefix sums of cnt, *total = their sum.  Each block
// takes the next partition from the counter, publishes its own sum, and wave 0
// looks back over 64 lower partitions at a time until it meets an inclusive
// sum; a partition only waits on partitions taken earlier, by running blocks.
__global__ void __launch_bounds__(kThreads) k_pair_offsets(int64_t n_all, const uint32_t* __restrict__ ndev,
                                                           const uint32_t* __restrict__ order,
                                                           const uint32_t* __restrict__ count,
                                                           uint32_t* __restrict__ cnt, uint32_t* __restrict__ offs,
                                                           uint32_t* __restrict__ total,
                                                           unsigned long long* __restrict__ state,
                                                           uint32_t* __restrict__ host_total)
{
    __shared__ uint32_t tile[kBlockItems + kBlockItems / 16];
    __shared__ uint32_t s_part, s_excl;
    unsigned long long* const look = state + 1;
    if (threadIdx.x == 0) s_part = (uint32_t)atomicAdd(state, 1ull);
    __syncthreads();
    const int64_t part = s_part;
    const int64_t n = dev_count(n_all, ndev);
    const int64_t base = part * kBlockItems;
#pragma unroll
    for (int i = 0; i < kItems; ++i) {
        const int k = i * kThreads + threadIdx.x;
        const int64_t idx = base + k;
        const uint32_t c = idx < n ? count[order[idx]] : 0u;
        tile[scan_pad(k)] = c;
        if (idx < n_all) cnt[idx] = c;
    }
    __syncthreads();
    uint32_t v[kItems];
    uint32_t sum = 0;
#pragma unroll
    for (int i = 0; i < kItems; ++i) {
        v[i] = tile[scan_pad(threadIdx.x * kItems + i)];
        sum = sat_add(sum, v[i]);
    }
    uint32_t tot;
    const uint32_t local = block_excl_scan(sum, &tot);
    if (threadIdx.x < 64) {
        const int lane = (int)threadIdx.x;
        if (lane == 0) store_agent64(look + part, (part == 0 ? kPsInc : kPsAgg) | tot);
        uint32_t excl = 0u;
        if (part > 0) {
            int64_t q = part - 1;
            for (;;) {  // partition 0 is inclusive, so this ends there at the latest
                const unsigned long long w = q - lane >= 0 ? load_agent64(look + (q - lane)) : kPsInc;
                const unsigned long long f = w & kPsFlags;
                const uint64_t incm = __ballot(f == kPsInc);
                const uint64_t unpub = __ballot(f == 0ull);
                const int fi = incm ? __builtin_ctzll(incm) : 64;
                const int fu = unpub ? __builtin_ctzll(unpub) : 64;
                // lanes [0, take) are published; with fu > fi they end at an inclusive sum
                const int take = fu > fi ? fi + 1 : fu;
                excl = sat_add(excl, wave_sum_sat(lane < take ? (uint32_t)w : 0u));
                if (fu > fi) break;
                q -= take;
                if (take == 0) __builtin_amdgcn_s_sleep(1);  // partition q is running and has not published yet
            }
            if (lane == 0) store_agent64(look + part, kPsInc | sat_add(excl, tot));
        }
        if (lane == 0) s_excl = excl;
    }
    __syncthreads();
    uint32_t run = sat_add(s_excl, local);
#pragma unroll
    for (int i = 0; i < kItems; ++i) {
        tile[scan_pad(threadIdx.x * kItems + i)] = run;
        run = sat_add(run, v[i]);
    }
    if (threadIdx.x == kThreads - 1 && base + kBlockItems >= n_all) {  // the last partition
        *total = run;
        if (host_total) *host_total = run;
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < kItems; ++i) {
        const int k = i * kThreads + threadIdx.x;
        if (base + k < n_all) offs[base + k] = tile[scan_pad(k)];
    }
}

void pair_offsets(const uint32_t* order, const uint32_t* count, Count n, uint32_t* cnt, uint32_t* offs,
                  uint32_t* total, uint32_t* state, hipStream_t s, uint32_t* host_total)
{
    if (n.cap <= 0) {
        launch_fill_u32(total, 0u, 1, s);
        if (host_total) launch_fill_u32(host_total, 0u, 1, s);
        return;
    }
    const int64_t nb = (n.cap + kBlockItems - 1) / kBlockItems;
    k_pair_offsets<<<(unsigned)nb, kThreads, 0, s>>>(n.cap, n.dev, order, count, cnt, offs, total,
                                                     reinterpret_cast<unsigned long long*>(state), host_total);
}

// ---------------------------------------------------------------------------
// Single-sweep radix sort
// ---------------------------------------------------------------------------

constexpr uint32_t kFlagAgg = 1u << 30;       // partition's own digit count published
constexpr uint32_t kFlagInc = 2u << 30;       // count including all lower partitions
constexpr uint32_t kCountMask = kFlagAgg - 1u;
constexpr int kMaxPasses = 4;
constexpr int kHistRep = kSortHistCopies;  // histogram copies (block b adds to copy b % 8): 8x less atomic contention
static_assert(kSortPassStride == kMaxPasses * kBins, "histogram copy stride");
constexpr int64_t kHistWords = (int64_t)kHistRep * kMaxPasses * kBins;
constexpr int64_t kStateBase = kHistWords + 64;  // words: histograms, counters, kept count

// Temp layout (uint32 words): [copy][pass][256] global digit counts, [pass]
// partition counters (at kHistWords), the kept count, then
// [pass][partition][256] look-back state.
int64_t sort_head_words() { return kStateBase; }
int64_t sort_state_words(int64_t cap) { return (int64_t)kMaxPasses * radix_blocks(cap) * kBins; }

__device__ __forceinline__ uint32_t load_agent(const uint32_t* p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void store_agent(uint32_t* p, uint32_t v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Digit counts of every pass over all n items (per-wave LDS histograms).  With
// drop, items whose key is kDropKey are left out and the number of the others
// is added to *kept.  Blocks count 1024-item chunks (4 per thread): the kernel
// is latency bound, and more, shorter blocks finish sooner than 4096-item ones
// (room depth sort 76 -> 71 us).
constexpr int kHistItems = 4;
constexpr int kHistBlockItems = kThreads * kHistItems;
__global__ void __launch_bounds__(kThreads) k_sort_hist(const uint32_t* __restrict__ keys, int64_t cap,
                                                        const uint32_t* __restrict__ ndev, int passes,
                                                        uint32_t* __restrict__ ghist, int drop,
                                                        uint32_t* __restrict__ kept, uint32_t* __restrict__ state,
                                                        int64_t state_stride, int64_t part_items)
{
    __shared__ uint32_t h[4][kMaxPasses][kBins];
    __shared__ uint32_t s_kept;
    const int64_t n = dev_count(cap, ndev);
    for (int i = threadIdx.x; i < 4 * kMaxPasses * kBins; i += kThreads) (&h[0][0][0])[i] = 0u;
    if (threadIdx.x == 0) s_kept = 0u;
    __syncthreads();
    const int w = threadIdx.x >> 6;
    uint32_t mine = 0u;
    // zero the passes' look-back words of the partitions they will use
    // (state_stride words per pass; the passes run after this kernel)
    {
        const int64_t words = ((n + part_items - 1) / part_items) * kBins;
        const int64_t gt = (int64_t)blockIdx.x * kThreads + threadIdx.x, gs = (int64_t)gridDim.x * kThreads;
        for (int p = 0; p < passes; ++p)
            for (int64_t i = gt; i < words; i += gs) state[(int64_t)p * state_stride + i] = 0u;
    }
    // each thread counts kHistItems keys per chunk, all loaded before any is
    // counted so that their latencies overlap; chunks are strided by the grid
    for (int64_t i0 = (int64_t)blockIdx.x * kHistBlockItems; i0 < n; i0 += (int64_t)gridDim.x * kHistBlockItems) {
    uint32_t key[kHistItems];
#pragma unroll
    for (int r = 0; r < kHistItems; ++r) {
        const int64_t i = i0 + (int64_t)r * kThreads + threadIdx.x;
        key[r] = i < n ? keys[i] : kDropKey;
    }
#pragma unroll
    for (int r = 0; r < kHistItems; ++r) {
        const int64_t i = i0 + (int64_t)r * kThreads + threadIdx.x;
        const uint32_t k = key[r];
        const bool valid = i < n && !(drop && k == kDropKey);
        const uint64_t active = __ballot(valid);
        if (active == 0ull) continue;
        if (valid) ++mine;
        const int first = __builtin_ctzll(active);
        for (int p = 0; p < passes; ++p) {
            const uint32_t d = (k >> (8 * p)) & 0xFFu;
            const uint32_t d0 = __shfl(d, first, 64);
            // skewed digits (e.g. the exponent byte of depths) are mostly one
            // value per wave: one lane adds them all instead of 64 conflicting atomics
            if (__ballot(valid && d != d0) == 0ull) {
                if (__lane_id() == (unsigned)first) atomicAdd(&h[w][p][d0], (uint32_t)__popcll(active));
            } else if (valid) {
                atomicAdd(&h[w][p][d], 1u);
            }
        }
    }
    }
    if (drop && mine) atomicAdd(&s_kept, mine);
    __syncthreads();
    for (int i = threadIdx.x; i < passes * kBins; i += kThreads) {
        const int p = i / kBins, b = i % kBins;
        const uint32_t c = h[0][p][b] + h[1][p][b] + h[2][p][b] + h[3][p][b];
        if (c) atomicAdd(&ghist[(int64_t)(blockIdx.x % kHistRep) * kMaxPasses * kBins + i], c);
    }
    if (drop && threadIdx.x == 0 && s_kept) atomicAdd(kept, s_kept);
}

// One digit pass.  ghist: this pass's 256 global counts in histogram copy 0
// (the other copies follow at a stride of kMaxPasses * 256); state: this
// pass's [partition][256] look-back words (zero on entry); counter: zero on entry.
template <int ITEMS>
__global__ void __launch_bounds__(kThreads) k_sort_pass(const uint32_t* __restrict__ keys_in,
                                                        const uint32_t* __restrict__ vals_in,
                                                        uint32_t* __restrict__ keys_out,
                                                        uint32_t* __restrict__ vals_out, int64_t cap,
                                                        const uint32_t* __restrict__ ndev, int shift,
                                                        const uint32_t* __restrict__ ghist, uint32_t* state,
                                                        uint32_t* counter, int drop)
{
    constexpr int BI = kThreads * ITEMS;  // partition
    constexpr int WI = BI / 4;            // per wave
    __shared__ uint32_t s_key[BI];
    __shared__ uint32_t s_val[BI];
    __shared__ uint32_t cnt[4][kBins];
    __shared__ uint32_t s_start[kBins];  // block-local first slot of each digit
    __shared__ uint32_t s_out[kBins];    // global position of that slot
    __shared__ uint32_t s_part;
    const int64_t n = dev_count(cap, ndev);
    // blocks take partitions in counter order until none is left, so the grid
    // need not match the (device-side) item count.  Blocks beyond the
    // partition count leave before touching the counter (with a generous
    // capacity most of the grid would otherwise queue on that one word just to
    // exit), so the first `parts` blocks take one partition each.
    const int64_t parts = (n + BI - 1) / BI;
    if ((int64_t)blockIdx.x >= parts) return;
    for (;;) {
    __syncthreads();  // the previous partition's LDS is no longer read
    if (threadIdx.x == 0) s_part = atomicAdd(counter, 1u);
    for (int i = threadIdx.x; i < 4 * kBins; i += kThreads) (&cnt[0][0])[i] = 0u;
    __syncthreads();
    const uint32_t part = s_part;
    const int64_t base = (int64_t)part * BI;
    if (base >= n) return;  // every partition above this one is empty too
    // this digit's global count (thread t = digit t), loaded early so its latency overlaps the ranking
    uint32_t gcount = 0u;
#pragma unroll
    for (int r = 0; r < kHistRep; ++r) gcount += ghist[(int64_t)r * kMaxPasses * kBins + threadIdx.x];
    const int w = threadIdx.x >> 6;
    const unsigned lane = __lane_id();
    const int64_t wbase = base + (int64_t)w * WI;
    const uint64_t lt = lanemask_lt();
    uint32_t key[ITEMS], val[ITEMS], rank[ITEMS];
#pragma unroll
    for (int r = 0; r < ITEMS; ++r) {
        const int64_t idx = wbase + r * 64 + lane;
        const bool valid = idx < n;
        key[r] = valid ? keys_in[idx] : 0u;
        val[r] = valid ? (vals_in ? vals_in[idx] : (uint32_t)idx) : 0u;
    }
    // stable rank of every item among the wave's items of its digit
#pragma unroll
    for (int r = 0; r < ITEMS; ++r) {
        const bool valid = wbase + r * 64 + lane < n && !(drop && key[r] == kDropKey);
        const uint64_t active = __ballot(valid);
        rank[r] = 0u;
        if (active == 0ull) continue;
        const uint32_t d = (key[r] >> shift) & 0xFFu;
        const uint32_t d0 = __shfl(d, __builtin_ctzll(active), 64);
        const uint64_t m = __ballot(valid && d != d0) == 0ull ? active : match8(d, active);
        const uint32_t before = valid ? cnt[w][d] : 0u;
        rank[r] = before + (uint32_t)__popcll(m & lt);
        if (valid && (m & lt) == 0ull) cnt[w][d] = before + (uint32_t)__popcll(m);
    }
    __syncthreads();
    const int d = threadIdx.x;  // one thread per digit from here
    const uint32_t c0 = cnt[0][d], c1 = cnt[1][d], c2 = cnt[2][d], c3 = cnt[3][d];
    const uint32_t bc = c0 + c1 + c2 + c3;
    store_agent(state + (int64_t)part * kBins + d, (part == 0 ? kFlagInc : kFlagAgg) | bc);
    cnt[0][d] = 0u;
    cnt[1][d] = c0;
    cnt[2][d] = c0 + c1;
    cnt[3][d] = c0 + c1 + c2;
    uint32_t tot;
    const uint32_t start = block_excl_scan(bc, &tot);
    // look back: sum this digit's counts over all lower partitions, reading
    // eight predecessors at a time (their loads are in flight together)
    uint32_t excl = 0u;
    if (part > 0) {
        constexpr int kWin = 8;
        int64_t q = (int64_t)part - 1;
        while (q >= 0) {  // partition 0 publishes an inclusive count, so this ends there at the latest
            uint32_t v[kWin];
#pragma unroll
            for (int i = 0; i < kWin; ++i) v[i] = q - i >= 0 ? load_agent(state + (q - i) * kBins + d) : kFlagInc;
            int used = 0;
            bool found = false;
#pragma unroll
            for (int i = 0; i < kWin; ++i) {
                if (found || used < i) continue;  // stop at the first inclusive or unpublished word
                const uint32_t flag = v[i] & ~kCountMask;
                if (flag == 0u) continue;
                excl += v[i] & kCountMask;
                ++used;
                found = flag == kFlagInc;
            }
            if (found) break;
            q -= used;
            if (used < kWin) __builtin_amdgcn_s_sleep(1);  // partition q has not published yet; it is running
        }
        store_agent(state + (int64_t)part * kBins + d, kFlagInc | (excl + bc));
    }
    uint32_t gtot;
    const uint32_t gstart = block_excl_scan(gcount, &gtot);
    s_start[d] = start;
    s_out[d] = gstart + excl;
    __syncthreads();
    // stage in digit order, then write runs out with consecutive addresses
#pragma unroll
    for (int r = 0; r < ITEMS; ++r) {
        if (wbase + r * 64 + lane < n && !(drop && key[r] == kDropKey)) {
            const uint32_t dd = (key[r] >> shift) & 0xFFu;
            const uint32_t li = s_start[dd] + cnt[w][dd] + rank[r];
            s_key[li] = key[r];
            s_val[li] = val[r];
        }
    }
    __syncthreads();
    const int m_items = (int)tot;  // items kept by this partition
    for (int i = threadIdx.x; i < m_items; i += kThreads) {
        const uint32_t k = s_key[i];
        const uint32_t dd = (k >> shift) & 0xFFu;
        const uint32_t pos = s_out[dd] + ((uint32_t)i - s_start[dd]);
        keys_out[pos] = k;
        vals_out[pos] = s_val[i];
    }
    if ((int64_t)gridDim.x >= parts) return;  // one partition per block: none left
    }
}

// Items per thread: from the capacity, or smaller partitions for an expected
// count below it when the look-back state has room for their number.
static int plan_items(int64_t cap, const SortTemp& t, int64_t size_hint)
{
    int items = sort_items(cap);
    if (size_hint > 0 && size_hint < cap && sort_items(size_hint) != items) {
        const int hi = sort_items(size_hint);
        if (t.state_words >= (int64_t)kMaxPasses * radix_blocks_items(cap, hi) * kBins) items = hi;
    }
    return items;
}

SortPrep radix_sort_prep(Count n, int end_bit, const SortTemp& t, int64_t size_hint)
{
    SortPrep p;
    if (n.cap <= 0 || n.cap > (int64_t)kCountMask) return p;
    const int items = plan_items(n.cap, t, size_hint);
    p.ghist = t.head;
    p.state = t.state;
    p.state_stride = (int64_t)radix_blocks_items(n.cap, items) * kBins;
    p.part_items = (int64_t)kThreads * items;
    p.passes = std::min(kMaxPasses, (end_bit + 7) / 8);
    return p;
}

int radix_sort_u32(uint32_t* keys, uint32_t* vals, bool identity_vals, Count n, int end_bit, const SortTemp& t,
                   hipStream_t s, const uint32_t** kept, const uint32_t* keys_src, int64_t size_hint, bool hist_done)
{
    if (kept) *kept = nullptr;
    if (n.cap <= 0) return 0;
    if (n.cap > (int64_t)kCountMask) return -1;  // counts share a word with the look-back flags
    const int items = plan_items(n.cap, t, size_hint);
    const int nb = radix_blocks_items(n.cap, items);
    const int passes = std::min(kMaxPasses, (end_bit + 7) / 8);
    uint32_t* ghist = t.head;  // histograms and counters: zero on entry
    uint32_t* counters = t.head + kHistWords;
    uint32_t* kept_dev = counters + kMaxPasses;
    uint32_t* state = t.state;  // the look-back words: zeroed by k_sort_hist
    const int drop = kept != nullptr;
    const int hb = (int)std::min<int64_t>(std::max<int64_t>(nb, (n.cap + kHistBlockItems - 1) / kHistBlockItems), 2048);
    // pass grid: blocks take partitions until none is left, so with an
    // expected count (capacity a generous bound) the grid follows it (with a
    // margin) rather than the capacity
    const int64_t grid_items = size_hint > 0 ? std::min<int64_t>(n.cap, size_hint + size_hint / 2 + 4096) : n.cap;
    const int pb = std::min(radix_blocks_items(grid_items, items), 2048);
    const uint32_t* first = keys_src ? keys_src : keys;
    if (!hist_done || drop)
        k_sort_hist<<<hb, kThreads, 0, s>>>(first, n.cap, n.dev, passes, ghist, drop, kept_dev, state,
                                            (int64_t)nb * kBins, (int64_t)kThreads * items);
    uint32_t* kb[2] = {keys, t.keys_alt};
    uint32_t* vb[2] = {vals, t.vals_alt};
    int cur = 0;
    for (int p = 0; p < passes; ++p) {
        // after a dropping first pass the later ones see only the kept items
        const uint32_t* nd = (p > 0 && drop) ? kept_dev : n.dev;
        auto pass = items == 8 ? k_sort_pass<8> : k_sort_pass<16>;
        pass<<<pb, kThreads, 0, s>>>(p == 0 ? first : kb[cur], identity_vals ? nullptr : vb[cur], kb[cur ^ 1],
                                     vb[cur ^ 1], n.cap, nd, 8 * p, ghist + p * kBins,
                                     state + (int64_t)p * nb * kBins, counters + p, p == 0 ? drop : 0);
        identity_vals = false;
        cur ^= 1;
    }
    if (kept) *kept = kept_dev;
    return cur;
}

}  // namespace vcgs
