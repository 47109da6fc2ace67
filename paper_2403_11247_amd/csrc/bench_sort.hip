// Stand-alone timing of the library's radix sort (the depth and tile sorts of
// the render path) against hipCUB's DeviceRadixSort on the same keys: 32-bit
// depth-like keys (binary32 bits of depths in [0.5, 8)) at several sizes, and
// 12-bit tile ids emitted per entry over a rectangle of a 75 x 43 tile grid
// (the 1200x680 image's tiles).  Both results are checked against a host stable
// sort.  Comparison only: the render path never calls hipCUB.
//
//     python -m paper_2403_11247_amd.build --sort-bench
//     paper_2403_11247_amd/bench_sort
#include <hip/hip_runtime.h>
#include <hipcub/hipcub.hpp>
#include <cstdio>
#include <cstdlib>
#include <vector>
#include <algorithm>
#include <random>
#include <cstring>
#include "internal.h"

#define CK(x) do { hipError_t e = (x); if (e != hipSuccess) { printf("HIP error %s at %d\n", hipGetErrorString(e), __LINE__); exit(1); } } while (0)

static void run(const char* name, const std::vector<uint32_t>& hk, int end_bit, int reps)
{
    const int64_t n = (int64_t)hk.size();
    uint32_t *k0, *k, *v, *ka, *va, *head, *state;
    CK(hipMalloc(&k0, n * 4)); CK(hipMalloc(&k, n * 4)); CK(hipMalloc(&v, n * 4));
    CK(hipMalloc(&ka, n * 4)); CK(hipMalloc(&va, n * 4));
    CK(hipMalloc(&head, vcgs::sort_head_words() * 4));
    CK(hipMalloc(&state, vcgs::sort_state_words(n) * 4));
    CK(hipMemcpy(k0, hk.data(), n * 4, hipMemcpyHostToDevice));
    vcgs::SortTemp t{ka, va, head, state};
    hipStream_t s; CK(hipStreamCreate(&s));
    hipEvent_t e0, e1; CK(hipEventCreate(&e0)); CK(hipEventCreate(&e1));
    // library sort (identity values, keys read from k0)
    float best = 1e9, sum = 0;
    int which = 0;
    for (int r = 0; r < reps + 3; ++r) {
        CK(hipMemsetAsync(head, 0, vcgs::sort_head_words() * 4, s));
        CK(hipEventRecord(e0, s));
        which = vcgs::radix_sort_u32(k, v, true, vcgs::Count{n, nullptr}, end_bit, t, s, nullptr, k0);
        CK(hipEventRecord(e1, s));
        CK(hipEventSynchronize(e1));
        float ms; CK(hipEventElapsedTime(&ms, e0, e1));
        if (r >= 3) { best = std::min(best, ms); sum += ms; }
    }
    // check
    std::vector<uint32_t> ok(n), ov(n);
    CK(hipMemcpy(ok.data(), which ? ka : k, n * 4, hipMemcpyDeviceToHost));
    CK(hipMemcpy(ov.data(), which ? va : v, n * 4, hipMemcpyDeviceToHost));
    std::vector<uint32_t> idx(n);
    for (int64_t i = 0; i < n; ++i) idx[i] = (uint32_t)i;
    const uint32_t mask = end_bit >= 32 ? 0xFFFFFFFFu : ((1u << end_bit) - 1u);
    std::stable_sort(idx.begin(), idx.end(), [&](uint32_t a, uint32_t b) { return (hk[a] & mask) < (hk[b] & mask); });
    int64_t bad = 0;
    for (int64_t i = 0; i < n; ++i) bad += ov[i] != idx[i];
    printf("%s n=%lld bits=%d  lib: best %.1f us avg %.1f us  mismatches %lld\n", name, (long long)n, end_bit,
           best * 1e3, sum / reps * 1e3, (long long)bad);
    // hipCUB
    size_t tb = 0;
    CK(hipcub::DeviceRadixSort::SortPairs(nullptr, tb, k0, k, v, va, (int)n, 0, end_bit, s));
    void* tmp; CK(hipMalloc(&tmp, tb));
    std::vector<uint32_t> iv(n);
    for (int64_t i = 0; i < n; ++i) iv[i] = (uint32_t)i;
    CK(hipMemcpy(v, iv.data(), n * 4, hipMemcpyHostToDevice));
    best = 1e9; sum = 0;
    for (int r = 0; r < reps + 3; ++r) {
        CK(hipEventRecord(e0, s));
        CK(hipcub::DeviceRadixSort::SortPairs(tmp, tb, k0, k, v, va, (int)n, 0, end_bit, s));
        CK(hipEventRecord(e1, s));
        CK(hipEventSynchronize(e1));
        float ms; CK(hipEventElapsedTime(&ms, e0, e1));
        if (r >= 3) { best = std::min(best, ms); sum += ms; }
    }
    CK(hipMemcpy(ov.data(), va, n * 4, hipMemcpyDeviceToHost));
    bad = 0;
    for (int64_t i = 0; i < n; ++i) bad += ov[i] != idx[i];
    printf("%s n=%lld bits=%d  hipcub: best %.1f us avg %.1f us  mismatches %lld\n", name, (long long)n, end_bit,
           best * 1e3, sum / reps * 1e3, (long long)bad);
    fflush(stdout);
    CK(hipFree(tmp)); CK(hipFree(k0)); CK(hipFree(k)); CK(hipFree(v)); CK(hipFree(ka)); CK(hipFree(va));
    CK(hipFree(head)); CK(hipFree(state));
    CK(hipStreamDestroy(s));
}

int main()
{
    std::mt19937 rng(7);
    std::uniform_real_distribution<float> ud(0.5f, 8.0f);
    for (int64_t n : {100000, 300490, 1000000, 3000000}) {
        std::vector<uint32_t> hk(n);
        for (auto& x : hk) { float d = ud(rng); memcpy(&x, &d, 4); }
        run("depth", hk, 32, 20);
    }
    // tile-like keys: each entry covers a rectangle of a 75 x 43 tile grid, emitted row-major
    for (int64_t ne : {300490, 520000}) {
        std::vector<uint32_t> hk;
        std::uniform_int_distribution<int> tx(0, 74), ty(0, 42), sz(1, 4);
        for (int64_t i = 0; i < ne; ++i) {
            const int x0 = tx(rng), y0 = ty(rng), w = sz(rng), h = sz(rng);
            for (int y = y0; y < std::min(43, y0 + h); ++y)
                for (int x = x0; x < std::min(75, x0 + w); ++x) hk.push_back((uint32_t)(y * 75 + x));
        }
        run("tile", hk, 12, 20);
    }
    return 0;
}
