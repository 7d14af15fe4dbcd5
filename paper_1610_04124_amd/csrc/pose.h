// pose.h -- ground model of one frame from that frame's own camera pose.
//
// The paper takes the ground slope and the horizon as known for each image
// (Sec. 3), so the ground model disparity of a row, f_ground = alpha (r -
// horizon) with alpha = baseline cos(pitch) / height, changes from frame to
// frame.  A handle's ground table (Eq. 4 per row and pixel disparity) and its
// diving / gravity thresholds are built for the handle's camera; a frame that
// brings its own pose gets both rebuilt on the device before its columns run
// (pose_tables_kernel), into a table area owned by the handle (per-frame
// path) or by the batch (one area per job).  The sky and object tables do not
// depend on the pose.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "stixels.h"

namespace stx {

// One frame's ground table to build.  Host-side FP64 values: alpha (the one
// transcendental of the pose, cos, is taken on the host) and the model
// constants that do not depend on the row.
struct PoseItem {
    float* G;               // [H][D] by top-down image row, 0 above the horizon
    int32_t* hi;            // [H] diving threshold per top-down row
    int32_t* lo;            // [H] gravity threshold per top-down row
    double alpha;           // ground slope, px of disparity per row
    double horizon;         // top-down horizon row (multiple of 1/256)
    double sigma_d;         // disparity noise
    double eps_g;           // ground sigma = sqrt(sigma_d^2 + (eps_g mu)^2)
    double d_range;         // outlier density support [0, d_range]
    double c_out;           // log(d_range) - log(p_out)
    double log_1mp;         // log(1 - p_out)
    double tau_dive, tau_grav;
    int32_t H, D, g;        // frame height, disparity bins, cost grid 2^-g
    int32_t sub;            // bins of 2^-sub px
};

// Checks a frame pose against a handle (horizon on the 1/256 grid, finite
// pitch with |pitch| < pi/2, the bottom row's ground disparity within [0, d_range]:
// then every ground cost is bounded by the handle's exactness check) and
// fills `it` for a frame of height H.  Returns STIXELS_OK or
// STIXELS_E_INVALID_ARG with the reason in *why.
int make_pose_item(const stixels_params& p, int D, const stixels_pose& pose, int H, float* G,
                   int32_t* hi, int32_t* lo, PoseItem* it, const char** why);

// Builds one frame's table (per-frame path), or n frames' tables from a
// device array of descriptors (batch), rows up to hmax.
hipError_t launch_pose_tables(const PoseItem& it, hipStream_t st);
hipError_t launch_pose_tables(const PoseItem* d_items, int n, int hmax, hipStream_t st);

}  // namespace stx
