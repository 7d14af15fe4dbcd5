// noalloc.hip -- stixels_compute_noalloc: one frame through the fused
// persistent kernel with its workspace (descriptor, task counter, task list
// and the per-workgroup scratch slots of the prefix tables) in a fixed
// device array of the library, for callers that cannot allocate device
// memory.  Nothing here calls hipMalloc or hipFree.
#include <algorithm>
#include <atomic>
#include <mutex>
#include <string>

#include "handle.h"
#include "job_desc.h"
#include "launch.h"
#include "noalloc.h"
#include "stixels.h"

namespace {

// One copy per GPU, held from the library's first use on that GPU until the
// process ends.  Host code never passes the name itself to a kernel: the
// device address comes from hipGetSymbolAddress (noalloc_setup).
static __device__ __align__(256) unsigned char scratch[stx::kNoAllocScratchBytes];

constexpr int kMaxDevices = 64;
std::atomic<void*> g_scratch_ptr[kMaxDevices];
std::mutex g_setup_mutex;

int set_err(stixels_handle* h, int code, const std::string& msg) {
    if (h) h->err = msg;
    return code;
}

}  // namespace

namespace stx {

hipError_t noalloc_setup(int device) {
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    if (g_scratch_ptr[device].load(std::memory_order_acquire)) return hipSuccess;
    std::lock_guard<std::mutex> lock(g_setup_mutex);
    if (g_scratch_ptr[device].load(std::memory_order_relaxed)) return hipSuccess;
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    if (cur != device) return hipErrorInvalidDevice;     // the device must be current
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!ptr) return hipErrorInvalidSymbol;
    g_scratch_ptr[device].store(ptr, std::memory_order_release);
    return hipSuccess;
}

}  // namespace stx

extern "C" int stixels_compute_noalloc(stixels_handle* h, const float* d_disparity, int32_t width,
                                       int32_t height, void* stream, const stixels_output* out) {
    using namespace stx;
    if (!h) return STIXELS_E_INVALID_ARG;
    if (!d_disparity || !out || !out->counts || !out->records || !out->total_cost ||
        !out->overflow)
        return set_err(h, STIXELS_E_INVALID_ARG, "null input or output pointer");
    if (width < h->s || width > h->Wmax)
        return set_err(h, STIXELS_E_INVALID_ARG, "width outside [stixel_width, max_width]");
    if (height < 1 || height > h->Hmax)
        return set_err(h, STIXELS_E_INVALID_ARG, "height outside [1, max_height]");
    if (out->capacity < 1)
        return set_err(h, STIXELS_E_INVALID_ARG, "output capacity must be >= 1");
    const int ncols = width / h->s;
    // the workspace must hold the frame's header, task list and at least one
    // scratch slot; with fewer slots than columns the persistent kernel runs
    // fewer workgroups, each taking several columns in turn
    if (persist::frame_fused_bytes(ncols, height, h->D, 1) > kNoAllocScratchBytes)
        return set_err(h, STIXELS_E_RANGE,
                       "frame too large for the fixed workspace of stixels_compute_noalloc");
    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess || cur != h->device)
        return set_err(h, STIXELS_E_INVALID_ARG, "the handle's device must be current");
    // set up by stixels_create on the handle's device; looked up here only
    // if that failed
    hipError_t e = noalloc_setup(cur);
    if (e != hipSuccess)
        return set_err(h, STIXELS_E_HIP, std::string("fixed workspace lookup failed: ") +
                                             hipGetErrorString(e));
    void* ws = g_scratch_ptr[cur].load(std::memory_order_acquire);
    const hipStream_t st = static_cast<hipStream_t>(stream);
    persist::JobDesc job = persist::make_job_desc(h, d_disparity, width, height, *out);
    const int waves = frame_waves(h->waves, height, ncols, h->num_cu);
    int grid = 0;
    e = persist::launch_frame_fused(job, ws, kNoAllocScratchBytes, waves, h->num_cu, st, &grid);
    if (e != hipSuccess)
        return set_err(h, STIXELS_E_HIP, std::string("kernel launch failed: ") + hipGetErrorString(e));
    return STIXELS_OK;
}
