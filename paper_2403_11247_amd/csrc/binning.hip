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

__global__ void __launch_bounds__(256) k_gather_counts(int64_t n, const uint32_t* __restrict__ order,
                                                       const uint32_t* __restrict__ count, uint32_t* __restrict__ out)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) out[k] = count[order[k]];
}

void launch_gather_counts(int64_t n, const uint32_t* order, const uint32_t* count, uint32_t* out, hipStream_t s)
{
    if (n <= 0) return;
    k_gather_counts<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(n, order, count, out);
}

// One block per 256 depth-ordered entries; its threads walk the block's
// output range with a stride of 256 (coalesced stores) and locate the owning
// entry of each position by binary search over the block's offsets.  Entry e
// belongs to view e / n and its pairs carry that view's global tile ids.
constexpr int kEmitG = 256;

__global__ void __launch_bounds__(kEmitG) k_emit_pairs(EmitTab tab, int64_t n_entries,
                                                       const uint32_t* __restrict__ order,
                                                       const uint32_t* __restrict__ offs,
                                                       const uint32_t* __restrict__ count,
                                                       const uint2* __restrict__ rect, uint32_t* __restrict__ tile_ids,
                                                       uint32_t* __restrict__ gids, int64_t cap,
                                                       const uint32_t* __restrict__ total,
                                                       uint32_t* __restrict__ overflow)
{
    __shared__ uint32_t s_off[kEmitG + 1];
    __shared__ uint32_t s_gid[kEmitG];
    __shared__ uint2 s_rect[kEmitG];
    const int64_t k0 = (int64_t)blockIdx.x * kEmitG;
    const int64_t k = k0 + threadIdx.x;
    const int m = (int)((n_entries - k0) < kEmitG ? (n_entries - k0) : kEmitG);
    if (blockIdx.x == 0 && threadIdx.x == 0 && overflow && total && (int64_t)*total > cap) *overflow = 1u;
    if (k < n_entries) {
        const uint32_t g = order[k];
        s_gid[threadIdx.x] = g;
        s_rect[threadIdx.x] = rect[g];
        s_off[threadIdx.x] = offs[k];
        if ((int)threadIdx.x == m - 1) s_off[m] = offs[k] + count[g];
    }
    __syncthreads();
    const uint32_t lo = s_off[0];
    const uint32_t hi = (int64_t)s_off[m] < cap ? s_off[m] : (uint32_t)cap;
    for (uint32_t p = lo + threadIdx.x; p < hi; p += kEmitG) {
        // largest j in [0, m) with s_off[j] <= p
        int a = 0, b = m - 1;
        while (a < b) {
            const int mid = (a + b + 1) >> 1;
            if (s_off[mid] <= p) a = mid; else b = mid - 1;
        }
        const uint32_t e = s_gid[a];
        const int v = (int)(e / (uint32_t)tab.n);
        const uint2 r = s_rect[a];
        const uint32_t tx0 = r.x & 0xFFFFu, ty0 = r.x >> 16, tx1 = r.y & 0xFFFFu;
        const uint32_t w = tx1 - tx0 + 1u;
        const uint32_t local = p - s_off[a];
        const uint32_t ty = ty0 + local / w, tx = tx0 + local % w;
        tile_ids[p] = tab.tile_base[v] + ty * (uint32_t)tab.tiles_x[v] + tx;
        gids[p] = e;
    }
}

void launch_emit_pairs(const EmitTab& t, int64_t n_entries, const uint32_t* order, const uint32_t* offs,
                       const uint32_t* count, const uint2* rect, uint32_t* tile_ids, uint32_t* gids, int64_t cap,
                       const uint32_t* total, uint32_t* overflow, hipStream_t s)
{
    if (n_entries <= 0) return;
    k_emit_pairs<<<(unsigned)((n_entries + kEmitG - 1) / kEmitG), kEmitG, 0, s>>>(
        t, n_entries, order, offs, count, rect, tile_ids, gids, cap, total, overflow);
}

// [start, end) of every tile's run in the tile-sorted pair list (ranges must
// be zero-filled beforehand so that empty tiles read [0, 0)).
__global__ void __launch_bounds__(256) k_tile_ranges(int64_t cap, const uint32_t* __restrict__ ndev,
                                                     const uint32_t* __restrict__ t, uint32_t n_tiles,
                                                     uint32_t* __restrict__ ranges)
{
    const int64_t P = ndev ? min((int64_t)*ndev, cap) : cap;
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P) return;
    const uint32_t cur = t[p];
    if (cur >= n_tiles) return;
    if (p == 0 || t[p - 1] != cur) ranges[2 * cur] = (uint32_t)p;
    if (p == P - 1 || t[p + 1] != cur) ranges[2 * cur + 1] = (uint32_t)(p + 1);
}

void launch_tile_ranges(Count P, const uint32_t* tile_sorted, uint32_t n_tiles, uint32_t* ranges, hipStream_t s)
{
    if (P.cap <= 0) return;
    k_tile_ranges<<<(unsigned)((P.cap + 255) / 256), 256, 0, s>>>(P.cap, P.dev, tile_sorted, n_tiles, ranges);
}

}  // namespace vcgs
