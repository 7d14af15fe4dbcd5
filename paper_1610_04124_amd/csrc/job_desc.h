// job_desc.h -- descriptor of one frame for the persistent fused kernel,
// filled on the host from a handle (camera model and resident tables), the
// frame's device input and its caller-owned output.
#pragma once

#include "batch_kernel.h"
#include "handle.h"
#include "launch.h"

namespace stx::persist {

inline JobDesc make_job_desc(const stixels_handle* h, const float* disp, int W, int H,
                             const stixels_output& out) {
    JobDesc d;
    d.disp = disp;
    d.sky = h->d_sky;
    d.ground = h->d_ground;
    d.object_t = h->d_object_t;
    d.object_df = h->d_object_df;
    d.fg_hi = h->d_fg_hi;
    d.fg_lo = h->d_fg_lo;
    d.counts = out.counts;
    d.records = reinterpret_cast<uint32_t*>(out.records);
    d.total = out.total_cost;
    d.overflow = out.overflow;
    d.W = W;
    d.H = H;
    d.s = h->s;
    d.ncols = W / h->s;
    d.D = h->D;
    d.vtop = ground_top(h->p.camera.horizon_row, H);
    d.reduce_mode = h->p.reduce_mode;
    d.sub = h->p.subpixel_log2;
    d.cap = out.capacity;
    d.prior = h->prior;
    d.phase = nullptr;
    return d;
}

// One frame's columns through the persistent fused kernel (the batched
// launch with a single job): a one-block staging kernel writes the job's
// descriptor, its task list (column t is task t) and a zero task counter
// into the workspace, then the persistent kernel runs with one scratch slot
// of slot_floats(h, D) floats per resident workgroup.  No host-to-device copy
// and no allocation.  Workspace layout (ws 256-byte aligned):
//   [0, 256)               descriptor
//   [256, 512)             task counter
//   [512, 512 + 8 ncols)   task list, rounded up to 256 bytes
//   then the scratch slots, and kTableGuardBytes left unused at the end.
// Returns the workgroups launched in *grid_out (0 on error).
hipError_t launch_frame_fused(const JobDesc& job, void* ws, size_t ws_bytes, int waves,
                              int num_cu, hipStream_t st, int* grid_out);

// Bytes of workspace a frame of ncols columns needs for `slots` scratch slots.
size_t frame_fused_bytes(int ncols, int H, int D, int slots);

}  // namespace stx::persist
