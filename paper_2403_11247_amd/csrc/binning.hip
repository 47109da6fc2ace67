// Tile binning: after the Gaussians are sorted by depth, every visible
// Gaussian emits one (tile id, Gaussian index) pair per tile of its rectangle,
// in depth order and row-major within the rectangle.  A stable sort of these
// pairs by tile id then yields, per tile, the Gaussians in (depth, index)
// order -- the same order as sorting (tile << 32 | depth bits, index).
#include "internal.h"

namespace vcgs {

__global__ void __launch_bounds__(256) k_fill_u32(uint32_t* __restrict__ p, uint32_t v, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void __launch_bounds__(256) k_fill_f32(float* __restrict__ p, float v, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

void launch_fill_u32(uint32_t* p, uint32_t v, int64_t n, hipStream_t s)
{
    if (n <= 0) return;
    k_fill_u32<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(p, v, n);
}

__global__ void __launch_bounds__(256) k_zero_u32(ZeroSegs z, int64_t total)
{
    zero_segs(z, total, (int64_t)blockIdx.x * blockDim.x + threadIdx.x, (int64_t)gridDim.x * blockDim.x);
}

void launch_zero_u32(const ZeroSegs& zin, hipStream_t s)
{
    ZeroSegs z = zin;
    const int64_t total = zero_segs_normalise(z);
    if (total <= 0) return;
    const int64_t blocks = std::min<int64_t>((total + 255) / 256, 4096);
    k_zero_u32<<<(unsigned)blocks, 256, 0, s>>>(z, total);
}

void launch_fill_f32(float* p, float v, int64_t n, hipStream_t s)
{
    if (n <= 0) return;
    k_fill_f32<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(p, v, n);
}

__global__ void __launch_bounds__(256) k_copy_u32(uint32_t* __restrict__ dst, const uint32_t* __restrict__ src,
                                                  int64_t cap, const uint32_t* __restrict__ ndev)
{
    const int64_t n = ndev ? min((int64_t)*ndev, cap) : cap;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = src[i];
}

void launch_copy_u32(uint32_t* dst, const uint32_t* src, Count n, hipStream_t s)
{
    if (n.cap <= 0) return;
    k_copy_u32<<<(unsigned)((n.cap + 255) / 256), 256, 0, s>>>(dst, src, n.cap, n.dev);
}

// Pair emission, balanced over the output: block c writes pairs
// [c * kChunk, (c + 1) * kChunk).  k_chunk_starts records, for every chunk, the
// depth-ordered entry that owns its first pair; the block then stages the
// entries from there up to the owner of the next chunk's first pair (offsets,
// Gaussian ids, rectangles) in LDS, and its
// threads stride over the chunk's pairs (coalesced stores), locating each
// pair's owner by binary search over the staged offsets.  Entry e belongs to
// view e / n, and its pairs carry that view's global tile ids, row-major
// within its rectangle.
constexpr int kEmitG = 256;
constexpr int kChunk = 2048;  // pairs per block
constexpr int kSpan = 1024;   // entries staged at a time
constexpr int kRun = 8;       // consecutive pairs per thread

__global__ void __launch_bounds__(256) k_chunk_starts(int64_t n_all, const uint32_t* __restrict__ nvis,
                                                      const uint32_t* __restrict__ offs,
                                                      const uint32_t* __restrict__ cnt, int64_t cap,
                                                      uint32_t* __restrict__ chunk_start)
{
    const int64_t n = nvis ? min((int64_t)*nvis, n_all) : n_all;
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const int64_t lo = offs[k], hi = min(lo + (int64_t)cnt[k], cap);
    for (int64_t c = (lo + kChunk - 1) / kChunk; c * kChunk < hi; ++c) chunk_start[c] = (uint32_t)k;
}

__global__ void __launch_bounds__(kEmitG) k_emit_pairs(EmitTab tab, int64_t n_all, const uint32_t* __restrict__ nvis,
                                                       const uint32_t* __restrict__ order,
                                                       const uint32_t* __restrict__ offs,
                                                       const uint32_t* __restrict__ cnt,
                                                       const uint2* __restrict__ rect,
                                                       const uint32_t* __restrict__ chunk_start,
                                                       uint32_t* __restrict__ tile_ids, uint32_t* __restrict__ gids,
                                                       int64_t cap, const uint32_t* __restrict__ total,
                                                       uint32_t* __restrict__ overflow, int vec, SortPrep sp)
{
    __shared__ uint32_t s_off[kSpan + 1];
    __shared__ uint32_t s_gid[kSpan];
    __shared__ uint2 s_rect[kSpan];
    const int64_t n = nvis ? min((int64_t)*nvis, n_all) : n_all;
    const int64_t P = min((int64_t)*total, cap);
    // sticky: the largest pair count of any pass that outgrew the buffers since the flag was cleared
    if (blockIdx.x == 0 && threadIdx.x == 0 && overflow && (int64_t)*total > cap) *overflow = max(*overflow, *total);
    // the tile sort's digit histograms of this block's pairs, and its look-back
    // words cleared, so that the sort needs no histogram launch of its own
    __shared__ uint32_t s_hist[kSortPassStride];
    const int hp = sp.ghist ? sp.passes : 0;  // uniform
    if (hp) {
        for (int i = threadIdx.x; i < hp * 256; i += kEmitG) s_hist[i] = 0u;
        const int64_t words = ((P + sp.part_items - 1) / sp.part_items) * 256;
        const int64_t gt = (int64_t)blockIdx.x * kEmitG + threadIdx.x, gs = (int64_t)gridDim.x * kEmitG;
        for (int q = 0; q < hp; ++q)
            for (int64_t i = gt; i < words; i += gs) sp.state[q * sp.state_stride + i] = 0u;
    }
    // chunks strided by the grid, so a generous capacity does not launch blocks that only exit
    for (int64_t c = blockIdx.x; c * kChunk < P; c += gridDim.x) {  // uniform
    const int64_t p0 = c * kChunk;
    const int64_t p1 = min(p0 + kChunk, P);
    int64_t kbase = chunk_start[c];
    // the chunk's pairs belong to entries up to the one owning the next chunk's first pair
    const int64_t kend = p1 < P ? min((int64_t)chunk_start[c + 1] + 1, n) : n;
    int64_t pcur = p0;
    while (pcur < p1 && kbase < kend) {  // uniform; every round consumes kSpan entries or ends the chunk
        const int S = (int)min((int64_t)kSpan, kend - kbase);
        for (int i = threadIdx.x; i < S; i += kEmitG) {
            const uint32_t g = order[kbase + i];
            s_gid[i] = g;
            s_rect[i] = rect[g];
            s_off[i] = offs[kbase + i];
            if (i == S - 1) s_off[S] = offs[kbase + i] + cnt[kbase + i];
        }
        __syncthreads();
        const int64_t pend = min(p1, (int64_t)s_off[S]);
        // kRun consecutive pairs per thread: one binary search for the first,
        // then the owner and its tile advance by increments (an owner's pairs
        // are its rectangle's tiles in row-major order)
        for (int64_t q0 = pcur + (int64_t)threadIdx.x * kRun; q0 < pend; q0 += (int64_t)kEmitG * kRun) {
            // largest j in [0, S) with s_off[j] <= q0
            int a = 0, b = S - 1;
            while (a < b) {
                const int mid = (a + b + 1) >> 1;
                if ((int64_t)s_off[mid] <= q0) a = mid; else b = mid - 1;
            }
            uint32_t e = s_gid[a], row = 0, tx0 = 0, tx1 = 0, tx = 0, ty = 0, tbase = 0;
            // the owner's tile of pair p (local index p - s_off[a])
            auto owner = [&](int64_t p) {
                e = s_gid[a];
                const int v = (int)(e / (uint32_t)tab.n);
                const uint2 r = s_rect[a];
                tx0 = r.x & 0xFFFFu;
                tx1 = r.y & 0xFFFFu;
                const uint32_t w = tx1 - tx0 + 1u, local = (uint32_t)(p - (int64_t)s_off[a]);
                ty = (r.x >> 16) + local / w;
                tx = tx0 + local % w;
                row = (uint32_t)tab.tiles_x[v];
                tbase = tab.tile_base[v];
            };
            owner(q0);
            uint32_t next = s_off[a + 1];  // a + 1 <= S: s_off[S] > q0
            uint32_t tt[kRun], gg[kRun];
#pragma unroll
            for (int i = 0; i < kRun; ++i) {
                const int64_t p = q0 + i;
                if (p < pend) {
                    if ((int64_t)next <= p) {
                        // the next owner with pairs starts exactly at p (owners without pairs share its offset)
                        do {
                            ++a;
                            next = s_off[a + 1];
                        } while ((int64_t)next <= p);
                        owner(p);
                    }
                    tt[i] = tbase + ty * row + tx;
                    gg[i] = e;
                    for (int q = 0; q < hp; ++q) atomicAdd(&s_hist[q * 256 + ((tt[i] >> (8 * q)) & 0xFFu)], 1u);
                    if (++tx > tx1) {
                        tx = tx0;
                        ++ty;
                    }
                }
            }
            if (vec && (q0 & (kRun - 1)) == 0 && q0 + kRun <= pend) {
#pragma unroll
                for (int i = 0; i < kRun; i += 4) {
                    *reinterpret_cast<uint4*>(tile_ids + q0 + i) = make_uint4(tt[i], tt[i + 1], tt[i + 2], tt[i + 3]);
                    *reinterpret_cast<uint4*>(gids + q0 + i) = make_uint4(gg[i], gg[i + 1], gg[i + 2], gg[i + 3]);
                }
            } else {
#pragma unroll
                for (int i = 0; i < kRun; ++i)
                    if (q0 + i < pend) {
                        tile_ids[q0 + i] = tt[i];
                        gids[q0 + i] = gg[i];
                    }
            }
        }
        __syncthreads();
        pcur = pend;
        kbase += S;
    }
    }
    if (hp) {
        __syncthreads();
        uint32_t* gh = sp.ghist + (int64_t)(blockIdx.x % kSortHistCopies) * kSortPassStride;
        for (int i = threadIdx.x; i < hp * 256; i += kEmitG) {
            const uint32_t c = s_hist[i];
            if (c) atomicAdd(gh + i, c);
        }
    }
}

bool launch_emit_pairs(const EmitTab& t, int64_t n_entries, const uint32_t* nvis, const uint32_t* order,
                       const uint32_t* offs, const uint32_t* cnt, const uint2* rect, uint32_t* chunk_start,
                       uint32_t* tile_ids, uint32_t* gids, int64_t cap, const uint32_t* total, uint32_t* overflow,
                       const SortPrep& sp, hipStream_t s, int64_t grid_items)
{
    if (n_entries <= 0 || cap <= 0) return false;
    k_chunk_starts<<<(unsigned)((n_entries + 255) / 256), 256, 0, s>>>(n_entries, nvis, offs, cnt, cap, chunk_start);
    // blocks stride over the chunks, so the grid follows the expected count when given
    const int64_t gi = grid_items > 0 ? std::min(cap, grid_items) : cap;
    const int64_t blocks = std::min<int64_t>((gi + kChunk - 1) / kChunk, 4096);
    // 16-byte stores of whole runs need 16-byte aligned outputs
    const int vec = ((reinterpret_cast<uintptr_t>(tile_ids) | reinterpret_cast<uintptr_t>(gids)) & 15u) == 0u;
    k_emit_pairs<<<(unsigned)blocks, kEmitG, 0, s>>>(
        t, n_entries, nvis, order, offs, cnt, rect, chunk_start, tile_ids, gids, cap, total, overflow, vec, sp);
    return true;
}

int64_t emit_chunk_words(int64_t cap) { return (cap + kChunk - 1) / kChunk + 1; }

// [start, end) of every tile's run in the tile-sorted pair list (ranges must
// be zero-filled beforehand so that empty tiles read [0, 0)).  A thread takes
// four consecutive pairs (one 16-byte load when the list is 16-byte aligned);
// the neighbours across thread boundaries come from the adjacent lanes, and
// only the wave's two edge lanes load one more id.
constexpr uint32_t kNoTile = 0xFFFFFFFFu;
__global__ void __launch_bounds__(256) k_tile_ranges(int64_t cap, const uint32_t* __restrict__ ndev,
                                                     const uint32_t* __restrict__ t, uint32_t n_tiles,
                                                     uint32_t* __restrict__ ranges, int vec)
{
    const int64_t P = ndev ? min((int64_t)*ndev, cap) : cap;
    const int lane = threadIdx.x & 63;
    // grid-stride over 1024-pair block chunks (uniform per block): a generous
    // capacity does not launch blocks that only exit
    for (int64_t base = (int64_t)blockIdx.x * 1024; base < P; base += (int64_t)gridDim.x * 1024) {
        const int64_t p0 = base + 4 * threadIdx.x;
        uint32_t v[4];
        if (vec && p0 + 3 < P) {
            const uint4 q = *reinterpret_cast<const uint4*>(t + p0);
            v[0] = q.x;
            v[1] = q.y;
            v[2] = q.z;
            v[3] = q.w;
        } else {
#pragma unroll
            for (int i = 0; i < 4; ++i) v[i] = p0 + i < P ? t[p0 + i] : kNoTile;
        }
        uint32_t prev = __shfl_up(v[3], 1, 64), next = __shfl_down(v[0], 1, 64);
        if (lane == 0) prev = (p0 > 0 && p0 - 1 < P) ? t[p0 - 1] : kNoTile;
        if (lane == 63) next = p0 + 4 < P ? t[p0 + 4] : kNoTile;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int64_t p = p0 + i;
            const uint32_t cur = v[i];
            if (p >= P || cur >= n_tiles) continue;
            const uint32_t left = i > 0 ? v[i - 1] : prev, right = i < 3 ? v[i + 1] : next;
            if (p == 0 || left != cur) ranges[2 * cur] = (uint32_t)p;
            if (p == P - 1 || right != cur) ranges[2 * cur + 1] = (uint32_t)(p + 1);
        }
    }
}

void launch_tile_ranges(Count P, const uint32_t* tile_sorted, uint32_t n_tiles, uint32_t* ranges, hipStream_t s,
                        int64_t grid_items)
{
    if (P.cap <= 0) return;
    const int64_t gi = grid_items > 0 ? std::min(P.cap, grid_items) : P.cap;  // grid-stride loop
    const int64_t blocks = std::min<int64_t>((gi + 1023) / 1024, 4096);
    const int vec = (reinterpret_cast<uintptr_t>(tile_sorted) & 15u) == 0u;
    k_tile_ranges<<<(unsigned)blocks, 256, 0, s>>>(P.cap, P.dev, tile_sorted, n_tiles, ranges, vec);
}

}  // namespace vcgs
