// The allocation-free K-pass render: rcp_render's chain engine on a scratch
// area that is part of the library's device code object, for callers that
// cannot allocate device memory (code under graph capture, tight serving
// loops).
//
// `scratch` is a file-scope device array of kScratchBytes.  Each GPU the
// library runs on holds its own copy, at its own address, from the moment
// the code object is loaded until the process ends.  Its address on a device
// is looked up once, with that device current, and kept per device; host code
// uses only that address (the array's name in host code is a host-side
// stand-in, not a device address).
//
// Layout:
//   [0, kViewBytes)               the one-entry view table of the launch
//   [kCountersOfs, +kCountersBytes) band counters (zeroed by the setup kernel
//                                 of every call)
//   [kOrderOfs, +kOrderBytes)     tile scores and the cost order of views of
//                                 up to kOrderTiles tiles (written before each
//                                 launch; larger views take the screen order)
//   [kSpillOfs, kScratchBytes)    traversal stack overflow, one column per
//                                 thread of the grid
// Every call on a GPU shares that GPU's array and leaves its contents behind:
// calls that overlap on one GPU (two streams, or two threads) race.
#include <mutex>

#include "traverse.hpp"

namespace rcp {
namespace {

constexpr size_t kScratchBytes = size_t(64) << 20;   // 64 MiB per GPU
constexpr size_t kCountersOfs = 4096;
constexpr size_t kCountersBytes = 4096;
constexpr size_t kOrderOfs = kCountersOfs + kCountersBytes;
constexpr size_t kOrderTiles = size_t(1) << 16;   // 1080p and 1440p frames, with their padding
constexpr size_t kOrderBytes = 2 * kOrderTiles * sizeof(uint32_t);
constexpr size_t kSpillOfs = kOrderOfs + kOrderBytes;

static_assert(kViewBytes <= kCountersOfs, "the view table fits before the counters");

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

// Device address of `scratch` on the current device, looked up on the first
// call there and kept in a fixed table (the lookup allocates nothing either).
constexpr int kMaxDevices = 64;

rcp_status scratch_address(void** out) {
    static std::mutex mu;
    static void* addr[kMaxDevices] = {};
    int dev = 0;
    RCP_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) {
        set_error("device %d is beyond the %d devices the allocation-free render supports", dev, kMaxDevices);
        return RCP_ERR_INVALID_ARGUMENT;
    }
    std::lock_guard<std::mutex> lk(mu);
    if (addr[dev]) {
        *out = addr[dev];
        return RCP_OK;
    }
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
        if (e != hipSuccess) return hip_status(e, "hipGetSymbolAddress(scratch)", __FILE__, __LINE__);
        set_error("hipGetSymbolAddress(scratch) returned NULL");
        return RCP_ERR_DEVICE;
    }
    addr[dev] = p;
    *out = p;
    return RCP_OK;
}

}  // namespace

rcp_status render_noalloc(rcp_scene* s, const Camera& cam, int W, int H, int K, const Disp& disp, float* out_images,
                          int32_t* out_ids, hipStream_t stream) {
    void* base = nullptr;
    RCP_TRY_STATUS(scratch_address(&base));
    static_assert(kFetchWords * sizeof(uint32_t) <= kCountersBytes, "band counters fit");
    Workspace w;
    w.external = true;
    w.view = base;
    w.counters = (uint32_t*)((char*)base + kCountersOfs);
    w.order = (uint32_t*)((char*)base + kOrderOfs);
    w.order_cap = kOrderBytes / sizeof(uint32_t);
    w.spill = (int32_t*)((char*)base + kSpillOfs);
    w.spill_cap = (kScratchBytes - kSpillOfs) / sizeof(int32_t);
    return render_chain_fixed(s, w, cam, W, H, K, disp, out_images, out_ids, stream);
}

}  // namespace rcp

extern "C" {

rcp_status rcp_render_noalloc(rcp_scene* scene, const rcp_camera* base_camera, int W, int H, int K,
                              const rcp_displacement* disp, float* out_images, int32_t* out_ids, void* hip_stream) {
    using namespace rcp;
    clear_error();
    rcp_status st = check_scene(scene);
    if (st) return st;
    Camera c;
    if ((st = check_camera(base_camera, c))) return st;
    if ((st = check_disp(disp))) return st;
    if ((st = check_size(W, H))) return st;
    if (K < 1 || K > kMaxPasses) {
        set_error("K = %d must be in [1, %d]", K, kMaxPasses);
        return RCP_ERR_INVALID_ARGUMENT;
    }
    if (!out_images) {
        set_error("out_images must not be NULL");
        return RCP_ERR_INVALID_ARGUMENT;
    }
    const Disp d{disp->lambda_eye, disp->lambda_dir, disp->z0, disp->mode};
    return render_noalloc(scene, c, W, H, K, d, out_images, out_ids, (hipStream_t)hip_stream);
}

uint64_t rcp_render_noalloc_scratch_bytes(void) { return rcp::kScratchBytes; }

}  // extern "C"
