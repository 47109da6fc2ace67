// Mask training step (paper Sec. 3.3, eq. (13)): the mask loss over the
// current view frustum and the pruning of a finished window.
//
// L_m = weight * mean over the Gaussians in the frustum of sigmoid(m); only
// those Gaussians get dL_m/dm = weight * sigmoid'(m) / N.  The sums are taken
// per block and then over blocks in block order (deterministic).
// Pruning keeps Gaussian g iff sigmoid(m_g) > eps and its hit count reaches
// min_hits, and lists the kept indices in order (a stable compaction by scan).
#include "internal.h"

namespace vcgs {

constexpr int kMaskThreads = 256;

int mask_loss_blocks(int64_t n) { return (int)std::max<int64_t>(1, (n + kMaskThreads - 1) / kMaskThreads); }

__device__ __forceinline__ float sigmoid_f(float x) { return 1.0f / (1.0f + __expf(-x)); }

// per block: (sum of sigmoid(m) over the frustum, number in the frustum)
__global__ void __launch_bounds__(kMaskThreads) k_mask_partials(int64_t n, const float* __restrict__ logit,
                                                                const uint32_t* __restrict__ count,
                                                                float* __restrict__ partial)
{
    __shared__ float ss[kMaskThreads];
    __shared__ float sc[kMaskThreads];
    const int64_t g = (int64_t)blockIdx.x * kMaskThreads + threadIdx.x;
    const bool in = g < n && (!count || count[g] > 0u);
    ss[threadIdx.x] = in ? sigmoid_f(logit[g]) : 0.0f;
    sc[threadIdx.x] = in ? 1.0f : 0.0f;
    __syncthreads();
    for (int w = kMaskThreads / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            ss[threadIdx.x] += ss[threadIdx.x + w];
            sc[threadIdx.x] += sc[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        partial[2 * blockIdx.x] = ss[0];
        partial[2 * blockIdx.x + 1] = sc[0];
    }
}

// one block: loss and the frustum size, in block order (sums in double)
__global__ void __launch_bounds__(kMaskThreads) k_mask_finish(const float* __restrict__ partial, int nb, float weight,
                                                              float* __restrict__ loss, float* __restrict__ inv_count)
{
    __shared__ double ss[kMaskThreads];
    __shared__ double sc[kMaskThreads];
    double a = 0.0, c = 0.0;
    for (int i = threadIdx.x; i < nb; i += kMaskThreads) {
        a += (double)partial[2 * i];
        c += (double)partial[2 * i + 1];
    }
    ss[threadIdx.x] = a;
    sc[threadIdx.x] = c;
    __syncthreads();
    for (int w = kMaskThreads / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            ss[threadIdx.x] += ss[threadIdx.x + w];
            sc[threadIdx.x] += sc[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double cnt = sc[0];
        if (loss) *loss = cnt > 0.0 ? (float)((double)weight * ss[0] / cnt) : 0.0f;
        *inv_count = cnt > 0.0 ? (float)(1.0 / cnt) : 0.0f;
    }
}

__global__ void __launch_bounds__(kMaskThreads) k_mask_grad(int64_t n, const float* __restrict__ logit,
                                                            const uint32_t* __restrict__ count, float weight,
                                                            const float* __restrict__ inv_count,
                                                            float* __restrict__ dl_dm)
{
    const int64_t g = (int64_t)blockIdx.x * kMaskThreads + threadIdx.x;
    if (g >= n || (count && count[g] == 0u)) return;
    const float s = sigmoid_f(logit[g]);
    dl_dm[g] += weight * s * (1.0f - s) * *inv_count;
}

void launch_mask_loss(int64_t n, const float* logit, const uint32_t* count, float weight, float* dl_dm, float* loss,
                      float* partial, hipStream_t s)
{
    if (n <= 0) {
        if (loss) launch_fill_f32(loss, 0.0f, 1, s);
        return;
    }
    const int nb = mask_loss_blocks(n);
    float* inv_count = partial + 2 * (int64_t)nb;
    k_mask_partials<<<nb, kMaskThreads, 0, s>>>(n, logit, count, partial);
    k_mask_finish<<<1, kMaskThreads, 0, s>>>(partial, nb, weight, loss, inv_count);
    if (dl_dm) k_mask_grad<<<nb, kMaskThreads, 0, s>>>(n, logit, count, weight, inv_count, dl_dm);
}

__global__ void __launch_bounds__(256) k_prune_flags(int64_t n, const float* __restrict__ logit, float thr,
                                                     const uint32_t* __restrict__ hits, uint32_t min_hits,
                                                     uint8_t* __restrict__ keep, uint32_t* __restrict__ flags)
{
    const int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (g >= n) return;
    const bool k = logit[g] > thr && (!hits || hits[g] >= min_hits);
    if (keep) keep[g] = k ? 1u : 0u;
    flags[g] = k ? 1u : 0u;
}

__global__ void __launch_bounds__(256) k_prune_scatter(int64_t n, const uint32_t* __restrict__ flags,
                                                       const uint32_t* __restrict__ offs,
                                                       uint32_t* __restrict__ kept_index)
{
    const int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (g < n && flags[g]) kept_index[offs[g]] = (uint32_t)g;
}

void launch_mask_prune(int64_t n, const float* logit, float thr, const uint32_t* hits, uint32_t min_hits,
                       uint8_t* keep, uint32_t* flags_tmp, uint32_t* offs_tmp, uint32_t* kept_index,
                       uint32_t* n_kept, uint32_t* scan_tmp, hipStream_t s)
{
    if (n <= 0) {
        launch_fill_u32(n_kept, 0u, 1, s);
        return;
    }
    const unsigned blocks = (unsigned)((n + 255) / 256);
    k_prune_flags<<<blocks, 256, 0, s>>>(n, logit, thr, hits, min_hits, keep, flags_tmp);
    exclusive_scan_u32(flags_tmp, offs_tmp, n, n_kept, scan_tmp, s);
    if (kept_index) k_prune_scatter<<<blocks, 256, 0, s>>>(n, flags_tmp, offs_tmp, kept_index);
}

}  // namespace vcgs
