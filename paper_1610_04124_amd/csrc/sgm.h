// sgm.h -- semi-global matching stage (census costs, four path directions)
// ahead of the stixel path: internal launch interface.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace stx::sgm {

// Device workspace of a matching handle, sized for max_frames frames of
// max_width x max_height: census words of both views, and the summed path
// costs S [frame][y][x][d] (uint16).
struct SgmWorkspace {
    uint64_t* cl = nullptr;
    uint64_t* cr = nullptr;
    uint16_t* S = nullptr;
};

struct PathArgs {
    const uint64_t* cl;
    const uint64_t* cr;
    uint16_t* S;
    float* disp;            // [frame][y][x], written by the last pass
    int W, H, D, P1, P2;
};

// Disparities per lane of a path wave for D disparities (D <= 64 DPL).
int dpl_of(int D);

// The whole stage over `frames` frames stored back to back ([frame][H][W]
// uint8 images, [frame][H][W] float disparity out); enqueued on st.
hipError_t launch_sgm(const uint8_t* left, const uint8_t* right, int W, int H, int frames,
                      const SgmWorkspace& ws, int D, int P1, int P2, float* disp, hipStream_t st);

}  // namespace stx::sgm
