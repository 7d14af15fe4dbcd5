// handle.h -- layout of a stixel handle (one camera model), shared by the
// per-frame entry points and the batched launch.
#pragma once

#include <string>
#include <vector>

#include "launch.h"
#include "pose.h"
#include "stixels.h"

struct stixels_handle {
    stixels_params p;
    int D = 0, Hmax = 0, Wmax = 0, s = 0, ncols_max = 0;
    int device = 0;
    int num_cu = 0;
    int waves = 0;          // waves per column of the recurrence (0 = automatic)
    int po_placement = 0;   // object prefix table of the recurrence: 0 auto, 1 HBM, 2 LDS
    int lds_per_block = 0;  // bytes
    int frame_path = 0;     // stixels_compute: 0 auto, 1 staged kernels, 2 one fused launch
    int object_lut = 0;     // staged table build: 0 offline object LUT, 1 online Eq. 4
    int last_path = 0;      // path of the last stixels_compute (1 or 2)
    size_t ws_bytes = 0;    // bytes of d_po (the fused path's whole workspace)
    stixels_batch* auto_batch = nullptr;   // batch object behind stixels_compute_batch
    // host copies of the rounded tables
    std::vector<float> sky, ground, object_t, object_df;
    std::vector<int32_t> fg_hi, fg_lo;
    std::vector<double> obj_k;   // per mean: Gaussian constant part, 2 sigma^2
    double c_out = 0.0;
    double* d_obj_k = nullptr;
    // device tables
    float* d_sky = nullptr;
    float* d_ground = nullptr;
    float* d_object_t = nullptr;
    float* d_object_df = nullptr;
    int32_t* d_fg_hi = nullptr;
    int32_t* d_fg_lo = nullptr;
    // per-frame workspace
    int16_t* d_q = nullptr;
    float* d_prefix = nullptr;
    int32_t* d_range = nullptr;
    float* d_po = nullptr;
    // the ground table and thresholds of the last frame with its own pose
    float* d_pose_ground = nullptr;    // [Hmax][D]
    int32_t* d_pose_hi = nullptr;      // [Hmax]
    int32_t* d_pose_lo = nullptr;      // [Hmax]
    bool pose_in_range = false;        // every valid pose keeps the grid arithmetic exact
    stx::Prior prior{};
    std::string err;
    int last_W = 0, last_H = 0;
};

// Device view of a handle's resident tables and priors.
inline stx::DeviceModel device_model(const stixels_handle* h) {
    stx::DeviceModel m{h->d_sky, h->d_ground, h->d_object_t, h->d_object_df, h->d_fg_hi,
                       h->d_fg_lo, h->D, h->Hmax, h->p.reduce_mode,
                       h->p.subpixel_log2, h->s,
                       h->p.camera.horizon_row, h->prior};
    m.obj_k = h->d_obj_k;
    m.c_out = h->c_out;
    m.object_online = h->object_lut;
    m.g = h->p.cost_grid_log2;
    return m;
}
