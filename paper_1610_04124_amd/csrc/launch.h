// launch.h -- host-side launchers of the per-frame and batched kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "internal.h"

namespace stx {

// Device-resident tables of one camera model (owned by a handle).
struct DeviceModel {
    const float* sky;       // [D]
    const float* ground;    // [max_height][D], top-down image rows
    const float* object_t;  // [D][D], row f: cost of pixel disparity d for mean f
    const float* object_df; // [D][D], row d: cost of pixel disparity d for every mean f
    const int32_t* fg_hi;   // [max_height], top-down image rows
    const int32_t* fg_lo;
    int D;
    int max_height;
    int reduce_mode;
    int sub;                // disparity bins of 2^-sub px
    int s;
    double horizon_row;
    Prior prior;
    // online object costs in the staged table build (Sec. 3.4 compares
    // them with the offline LUT): per mean the constant part and 2 sigma^2
    const double* obj_k = nullptr;
    double c_out = 0.0;
    int object_online = 0;
    int g = 0;
};

// Per-frame workspace views.
struct FrameWorkspace {
    int16_t* q;        // [ncols][H]
    float* prefix;     // [4][ncols][H+1]
    int32_t* range;    // [ncols][2]
    float* po;         // [ncols][D][H+1]
};

struct FrameOutput {
    int32_t* counts;
    uint32_t* records;   // [ncols][cap][3]
    float* total;
    uint8_t* overflow;
    int cap;
};

hipError_t launch_reduce(const DeviceModel& m, const float* disp, int W, int H, int ncols,
                         int16_t* q, hipStream_t st);
hipError_t launch_tables(const DeviceModel& m, const FrameWorkspace& ws, int H, int ncols,
                         int vtop, hipStream_t st);
// Waves per column of the per-frame recurrence: `requested` (1, 2 or 4,
// capped by the slot count) or, for 0, an automatic choice.
int frame_waves(int requested, int H, int ncols, int num_cu);
// Whether the per-frame recurrence tries the LDS copy of the object prefix
// table: placement 0 automatic, 1 never (HBM), 2 wherever it fits.
bool frame_po_lds(int placement, int H);
// lds_per_block: the device's LDS limit per workgroup (bytes).
hipError_t launch_dp(const DeviceModel& m, const FrameWorkspace& ws, int H, int ncols, int vtop,
                     int waves, bool po_lds, int lds_per_block, const FrameOutput& out,
                     hipStream_t st);
hipError_t run_selftest_mean(int D, int max_height, int64_t* mismatches);

// Bottom-up row limit of ground stixels for a frame of height H (FP64, the
// same reading the tables use: rows v with v <= floor(H-1-horizon_row)).
int ground_top(double horizon_row, int H);

}  // namespace stx
