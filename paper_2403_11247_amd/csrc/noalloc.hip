// Forward render of one view that allocates no device memory: every buffer of
// the pass (projected splats, depth and tile sorts, pair lists, tile ranges,
// per-pixel final transmittance and contributor counts) is carved out of one
// file-scope device array.  The kernels are those of vcgs_render_forward; only
// where their buffers come from differs.
//
// Each device that runs the library holds its own copy of the array, at its
// own address, from the first context created on it until the process ends.
// The host never passes the array's name to a kernel (in host code it is only
// a stand-in for the symbol): vcgs_create looks the device address up once per
// device and every launch takes that address.
#include <mutex>

#include "frame.h"

using namespace vcgs;

namespace {

constexpr size_t kNoAllocBytes = VCGS_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

std::mutex g_scratch_mu;
unsigned char* g_scratch_ptr[kMaxDevices] = {};  // device address of `scratch` per device

unsigned char* scratch_of(int device)
{
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    return (device >= 0 && device < kMaxDevices) ? g_scratch_ptr[device] : nullptr;
}

// Bump allocation inside the array: 256-byte aligned pieces; `used` keeps
// counting past the end so that the caller can report what a pass needs.
struct Carve {
    unsigned char* base;
    size_t used = 0;
    explicit Carve(unsigned char* b) : base(b) {}
    bool fits() const { return used <= kNoAllocBytes; }
    template <class T>
    T* get(int64_t count)
    {
        const size_t bytes = ((size_t)std::max<int64_t>(count, 1) * sizeof(T) + 255) & ~size_t(255);
        const size_t at = used;
        used += bytes;
        return used <= kNoAllocBytes ? reinterpret_cast<T*>(base + at) : nullptr;
    }
};

}  // namespace

namespace vcgs {

// Looks up this device's address of the array (the device must be current).
// Called by vcgs_create; later calls for the same device return at once.
int noalloc_init(int device)
{
    if (device < 0 || device >= kMaxDevices) return fail(VCGS_E_UNSUPPORTED, "device index above 63");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_ptr[device]) return VCGS_OK;
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
        return fail(VCGS_E_HIP, std::string("scratch symbol lookup failed: ") + hipGetErrorString(e));
    g_scratch_ptr[device] = static_cast<unsigned char*>(p);
    return VCGS_OK;
}

}  // namespace vcgs

extern "C" {

int vcgs_render_forward_noalloc(vcgs_ctx* ctx, const vcgs_gaussians* g, const vcgs_camera* cam,
                                const vcgs_pose* pose, const float bg[3], vcgs_images* out, void* stream)
{
    if (!ctx) return fail(VCGS_E_INVALID, "ctx is NULL");
    int rc;
    if ((rc = check_gaussians(g, 1)) != VCGS_OK) return rc;
    if ((rc = check_camera(cam)) != VCGS_OK) return rc;
    if (!pose || !bg || !out || !out->color || !out->depth || !out->alpha)
        return fail(VCGS_E_INVALID, "pose, bg or an output image is NULL");
    unsigned char* base = scratch_of(ctx->device);
    if (!base) return fail(VCGS_E_HIP, "scratch array of this device was not looked up");
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(hipSetDevice(ctx->device));

    Frame f;
    build_tables(1, g->n, cam, pose, bg, f);
    const int64_t HW = (int64_t)cam->width * cam->height;
    Carve cv(base);
    f.pt_dev = cv.get<ProjTab>(1);
    f.rec = cv.get<Splat>(f.E);
    f.depth_key = cv.get<uint32_t>(f.E);
    f.rect = cv.get<uint2>(f.E);
    f.count = cv.get<uint32_t>(f.E);
    f.ranges = cv.get<uint32_t>(2 * (int64_t)f.total_tiles);
    f.vt.t_final[0] = cv.get<float>(HW);
    f.vt.n_contrib[0] = cv.get<uint32_t>(HW);
    f.vt.color[0] = out->color;
    f.vt.depth[0] = out->depth;
    f.vt.alpha[0] = out->alpha;
    Work w{};
    alloc_work_e(w, f.E, [&](int64_t c) { return cv.get<uint32_t>(c); });
    if (!cv.fits())
        return fail(VCGS_E_CAPACITY, "the Gaussians and pixels need " + std::to_string(cv.used) +
                                         " bytes of scratch before the pairs; the array holds " +
                                         std::to_string(kNoAllocBytes));
    // the projection takes the table as a kernel argument (forward only: no device copy is read)
    f.tab_by_value = true;
    const uint32_t* ord = nullptr;
    // the pair scan also writes the pair count into the pinned word: no copy before the synchronisation
    if (f.E > 0) ord = phase_a(ctx->prof, *g, f, w, s, false, ctx->host_u32);
    else zero_pass(f, w, s);
    int64_t P = 0;
    if (f.E > 0) {
        HIP_TRY(hipStreamSynchronize(s));
        P = ctx->host_u32[0];
        if (P > kMaxSortItems) return fail(VCGS_E_UNSUPPORTED, "more than 2^30-1 (tile, Gaussian) pairs");
    }
    f.cap = P;
    f.gids = cv.get<uint32_t>(P);
    if (P > 0) alloc_work_p(w, P, [&](int64_t c) { return cv.get<uint32_t>(c); });
    if (!cv.fits()) {
        ctx->last_required_pairs = P;
        return fail(VCGS_E_CAPACITY, std::to_string(P) + " (tile, Gaussian) pairs take the pass to " +
                                         std::to_string(cv.used) + " bytes of scratch; the array holds " +
                                         std::to_string(kNoAllocBytes));
    }
    phase_b(ctx->prof, f, w, ord, s);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(VCGS_E_HIP, std::string("kernel launch failed: ") + hipGetErrorString(e));
    return VCGS_OK;
}

}  // extern "C"
