// pose.hip -- per-frame ground tables from the frame's own camera pose
// (Sec. 3: slope and horizon known for each image; Eq. 4 for the ground
// class; Sec. 3.4 for the table and the cost grid).
#include <cmath>

#include "launch.h"
#include "pose.h"

namespace stx {

namespace {

__device__ double normal_cdf(double x) { return 0.5 * erfc(-x / sqrt(2.0)); }

// Row r of one frame: the ground model disparity mu = alpha (r - horizon),
// the Gaussian of Eq. 4 with sigma = sqrt(sigma_d^2 + (eps_g mu)^2)
// truncated to [0, d_range], min with the outlier cost, rounded to the
// grid; 0 above the horizon (a ground stixel never reaches those rows).  The
// row's constant part (mass and normalisation) is evaluated once, by the
// first thread, in the same order of operations as the host tables.
__device__ void pose_row(const PoseItem& it, int r) {
    __shared__ double k_mu, k_2s2, k_c;
    __shared__ int k_ground;
    if (threadIdx.x == 0) {
        const double mu = it.alpha * ((double)r - it.horizon);
        const bool gr = (double)r >= it.horizon;
        if (gr) {
            const double e = it.eps_g * mu;
            const double sg = sqrt(it.sigma_d * it.sigma_d + e * e);
            const double mass = normal_cdf((it.d_range - mu) / sg) - normal_cdf(-mu / sg);
            k_c = log(mass) + log(sg * sqrt(2.0 * M_PI)) - it.log_1mp;
            k_2s2 = 2.0 * sg * sg;
        }
        k_mu = mu;
        k_ground = gr ? 1 : 0;
        const double hi = floor(ldexp(mu + it.tau_dive, it.sub));
        const double lo = ceil(ldexp(mu - it.tau_grav, it.sub));
        it.hi[r] = (int32_t)hi;
        it.lo[r] = (int32_t)lo;
    }
    __syncthreads();
    const double mu = k_mu;
    for (int d = threadIdx.x; d < it.D; d += blockDim.x) {
        float v = 0.0f;
        if (k_ground) {
            const double x = ldexp((double)d, -it.sub);
            const double gs = k_c + (x - mu) * (x - mu) / k_2s2;
            double c = it.c_out;
            if (isfinite(gs) && gs < c) c = gs;
            v = (it.g >= 0) ? (float)ldexp(rint(ldexp(c, it.g)), -it.g) : (float)c;
        }
        it.G[(size_t)r * it.D + d] = v;
    }
}

__global__ __launch_bounds__(256) void pose_one_kernel(PoseItem it) {
    if ((int)blockIdx.x < it.H) pose_row(it, (int)blockIdx.x);
}

__global__ __launch_bounds__(256) void pose_batch_kernel(const PoseItem* __restrict__ items) {
    const PoseItem it = items[blockIdx.y];
    if ((int)blockIdx.x < it.H) pose_row(it, (int)blockIdx.x);
}

}  // namespace

int make_pose_item(const stixels_params& p, int D, const stixels_pose& pose, int H, float* G,
                   int32_t* hi, int32_t* lo, PoseItem* it, const char** why) {
    const stixels_camera& c = p.camera;
    const stixels_model& m = p.model;
    if (!std::isfinite(pose.horizon_row) || std::fabs(pose.horizon_row) > 1048576.0 ||
        std::ldexp(pose.horizon_row, 8) != std::rint(std::ldexp(pose.horizon_row, 8))) {
        *why = "pose horizon_row must be a multiple of 1/256 with |horizon_row| <= 2^20";
        return STIXELS_E_INVALID_ARG;
    }
    // |pitch| < pi/2: the camera sees the ground plane from above (at pi/2
    // the double nearest pi/2 still has cos > 0, a slope of ~1e-17 px/row)
    const double cp = std::cos(pose.pitch_rad);
    if (!(std::fabs(pose.pitch_rad) < M_PI_2) || !(cp > 0.0)) {
        *why = "pose pitch must be finite with |pitch| < pi/2";
        return STIXELS_E_INVALID_ARG;
    }
    const double alpha = c.baseline_m * cp / c.cam_height_m;
    const double d_range = (double)p.max_disparity;
    // the largest ground model disparity of the frame (bottom row)
    const double mu_bottom = alpha * ((double)(H - 1) - pose.horizon_row);
    if (!(mu_bottom <= d_range)) {
        *why = "pose puts the ground disparity of the bottom row above max_disparity";
        return STIXELS_E_INVALID_ARG;
    }
    it->G = G;
    it->hi = hi;
    it->lo = lo;
    it->alpha = alpha;
    it->horizon = pose.horizon_row;
    it->sigma_d = m.sigma_disp;
    it->eps_g = m.ground_slope_noise;
    it->d_range = d_range;
    it->c_out = std::log(d_range) - std::log(m.p_out);
    it->log_1mp = std::log(1.0 - m.p_out);
    it->tau_dive = m.diving_tol_px;
    it->tau_grav = m.gravity_tol_px;
    it->H = H;
    it->D = D;
    it->g = p.cost_grid_log2;
    it->sub = p.subpixel_log2;
    return STIXELS_OK;
}

hipError_t launch_pose_tables(const PoseItem& it, hipStream_t st) {
    hipLaunchKernelGGL(pose_one_kernel, dim3((unsigned)it.H), dim3(256), 0, st, it);
    return hipGetLastError();
}

hipError_t launch_pose_tables(const PoseItem* d_items, int n, int hmax, hipStream_t st) {
    if (n < 1) return hipSuccess;
    hipLaunchKernelGGL(pose_batch_kernel, dim3((unsigned)hmax, (unsigned)n), dim3(256), 0, st,
                       d_items);
    return hipGetLastError();
}

}  // namespace stx
