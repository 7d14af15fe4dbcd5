// api.hip -- C ABI of the stixel library: handle creation (offline tables of
// Sec. 3.4 built in FP64 on the host, rounded to the cost grid, made resident
// in HBM), the per-frame compute entry point and the debug exports.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "handle.h"
#include "job_desc.h"
#include "launch.h"
#include "noalloc.h"
#include "stixels.h"

using namespace stx;

namespace {

int fail(stixels_handle* h, int code, const std::string& msg) {
    if (h) h->err = msg;
    return code;
}

// ------------------------------------------------------------------ Eq. 4
double gauss_cdf(double x) { return 0.5 * std::erfc(-x / std::sqrt(2.0)); }

// Per-pixel data cost of disparity d against a model disparity mu with
// standard deviation sigma: the min of the uniform-outlier cost and the
// Gaussian cost, the Gaussian normalised by its mass on [0, d_range].
double pixel_cost(double d, double mu, double sigma, double p_out, double d_range) {
    const double c_out = std::log(d_range) - std::log(p_out);
    const double mass = gauss_cdf((d_range - mu) / sigma) - gauss_cdf(-mu / sigma);
    const double g = std::log(mass) + std::log(sigma * std::sqrt(2.0 * M_PI)) -
                     std::log(1.0 - p_out) + (d - mu) * (d - mu) / (2.0 * sigma * sigma);
    if (!std::isfinite(g)) return c_out;
    return g < c_out ? g : c_out;
}

// Rounding onto the 2^-g cost grid; g < 0 keeps the value (costs off the grid).
double to_grid(double x, int g) {
    if (g < 0 || !std::isfinite(x)) return x;
    return std::ldexp(std::rint(std::ldexp(x, g)), -g);
}

bool finite_nonneg(double x) { return std::isfinite(x) && x >= 0.0; }

int validate(const stixels_params* p, std::string& why) {
    const stixels_camera& c = p->camera;
    const stixels_model& m = p->model;
    auto bad = [&](const char* w) { why = w; return STIXELS_E_INVALID_ARG; };
    if (!(c.focal_px > 0 && c.baseline_m > 0 && c.cam_height_m > 0 &&
          std::fabs(c.pitch_rad) < M_PI_2))
        return bad("camera focal, baseline and height must be > 0, |pitch| < pi/2");
    if (!std::isfinite(c.horizon_row) || std::fabs(c.horizon_row) > 1048576.0 ||
        std::ldexp(c.horizon_row, 8) != std::rint(std::ldexp(c.horizon_row, 8)))
        return bad("horizon_row must be a multiple of 1/256 with |horizon_row| <= 2^20");
    if (!(m.p_out > 0 && m.p_out < 1)) return bad("p_out must lie in (0, 1)");
    if (!(m.sigma_disp > 0 && m.sigma_sky > 0 && std::isfinite(m.sigma_disp) &&
          std::isfinite(m.sigma_sky)))
        return bad("sigma_disp and sigma_sky must be finite and > 0");
    if (!finite_nonneg(m.ground_slope_noise) || !finite_nonneg(m.object_depth_extent_m))
        return bad("ground_slope_noise and object_depth_extent_m must be finite and >= 0");
    if (!finite_nonneg(m.bic_cost) || !finite_nonneg(m.ordering_cost) ||
        !finite_nonneg(m.gravity_cost) || !finite_nonneg(m.diving_cost) ||
        !finite_nonneg(m.gravity_tol_px) || !finite_nonneg(m.diving_tol_px) ||
        m.ordering_tol_px < 0)
        return bad("prior costs and tolerances must be finite and >= 0");
    for (int a = 0; a < 3; ++a) {
        if (!finite_nonneg(m.first_cost[a])) return bad("first_cost must be finite and >= 0");
        for (int b = 0; b < 3; ++b) {
            const double t = m.trans_cost[a][b];
            if (!(t >= 0.0)) return bad("trans_cost must be >= 0 (INFINITY = forbidden)");
        }
        if (!std::isfinite(m.trans_cost[a][STIXELS_OBJECT]))
            return bad("trans_cost[*][object] must be finite");
    }
    if (p->stixel_width < 1 || p->stixel_width > kMaxStixelWidth)
        return bad("stixel_width must lie in 1..16");
    if (p->max_disparity < 2 || p->max_disparity > kMaxDisparity)
        return bad("max_disparity must lie in 2..256");
    if (p->max_height < 1 || p->max_height > kMaxHeight) return bad("max_height must lie in 1..1024");
    if (p->max_width < p->stixel_width) return bad("max_width must be >= stixel_width");
    if (p->max_stixels_per_column < 0) return bad("max_stixels_per_column must be >= 0");
    if (p->reduce_mode != 0 && p->reduce_mode != 1) return bad("reduce_mode must be 0 or 1");
    if (p->cost_grid_log2 < -1 || p->cost_grid_log2 > 12)
        return bad("cost_grid_log2 must lie in 0..12, or be -1 (costs off the grid)");
    if (p->flags & ~STIXELS_FLAG_BATCH_ONLY) return bad("unknown bits in flags");
    if (p->subpixel_log2 < 0 || p->subpixel_log2 > 3) return bad("subpixel_log2 must lie in 0..3");
    if ((p->max_disparity << p->subpixel_log2) > kMaxDisparity)
        return bad("max_disparity * 2^subpixel_log2 (disparity bins) must not exceed 256");
    if ((long long)p->max_height * (p->max_disparity << p->subpixel_log2) > (1LL << 20)) {
        why = "max_height * disparity bins must not exceed 2^20 (rounded-mean division bound)";
        return STIXELS_E_RANGE;
    }
    return STIXELS_OK;
}

template <typename T>
int upload(stixels_handle* h, T** dst, const std::vector<T>& src) {
    if (hipMalloc(reinterpret_cast<void**>(dst), src.size() * sizeof(T)) != hipSuccess)
        return fail(h, STIXELS_E_NOMEM, "hipMalloc of a table failed");
    if (hipMemcpy(*dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice) != hipSuccess)
        return fail(h, STIXELS_E_HIP, "hipMemcpy of a table failed");
    return STIXELS_OK;
}

void release(stixels_handle* h) {
    (void)hipFree(h->d_sky);
    (void)hipFree(h->d_ground);
    (void)hipFree(h->d_object_t);
    (void)hipFree(h->d_object_df);
    (void)hipFree(h->d_fg_hi);
    (void)hipFree(h->d_fg_lo);
    (void)hipFree(h->d_q);
    (void)hipFree(h->d_prefix);
    (void)hipFree(h->d_range);
    (void)hipFree(h->d_po);
    (void)hipFree(h->d_pose_ground);
    (void)hipFree(h->d_pose_hi);
    (void)hipFree(h->d_pose_lo);
    (void)hipFree(h->d_obj_k);
}

// Offline tables (Sec. 3.4) in FP64, rounded to the grid and stored as FP32.
int build_tables(stixels_handle* h) {
    const stixels_params& p = h->p;
    const stixels_model& m = p.model;
    // D disparity bins of 2^-k px (k = subpixel_log2); Eq. 4 is evaluated at
    // the bins' disparities in px, the outlier density stays uniform over
    // [0, max_disparity] px
    const int D = h->D, Hmax = h->Hmax, g = p.cost_grid_log2, k = p.subpixel_log2;
    const double dr = (double)p.max_disparity;
    auto px = [k](int i) { return std::ldexp((double)i, -k); };
    const double hr = p.camera.horizon_row;
    const double alpha = p.camera.baseline_m * std::cos(p.camera.pitch_rad) / p.camera.cam_height_m;
    double cmax = 0.0;
    auto keep = [&](double v) {
        cmax = std::fmax(cmax, std::fabs(v));
        return (float)v;
    };
    h->sky.resize(D);
    for (int d = 0; d < D; ++d)
        h->sky[d] = keep(to_grid(pixel_cost(px(d), 0.0, m.sigma_sky, m.p_out, dr), g));
    // ground rows by top-down image row r: model disparity alpha (r - horizon),
    // zero (never used) above the horizon
    h->ground.assign((size_t)Hmax * D, 0.0f);
    h->fg_hi.resize(Hmax);
    h->fg_lo.resize(Hmax);
    for (int r = 0; r < Hmax; ++r) {
        const double mu = alpha * ((double)r - hr);
        if ((double)r >= hr) {
            const double e = m.ground_slope_noise * mu;
            const double sg = std::sqrt(m.sigma_disp * m.sigma_disp + e * e);
            for (int d = 0; d < D; ++d)
                h->ground[(size_t)r * D + d] = keep(to_grid(pixel_cost(px(d), mu, sg, m.p_out, dr), g));
        }
        // thresholds in bins
        h->fg_hi[r] = (int32_t)std::floor(std::ldexp(mu + m.diving_tol_px, k));
        h->fg_lo[r] = (int32_t)std::ceil(std::ldexp(mu - m.gravity_tol_px, k));
    }
    // object table stored as [f][d]: one row per model mean f; beside it the
    // part of Eq. 4 that depends on the mean only (for online evaluation)
    h->object_t.resize((size_t)D * D);
    h->obj_k.resize((size_t)2 * D);
    h->c_out = std::log(dr) - std::log(m.p_out);
    for (int f = 0; f < D; ++f) {
        const double e = px(f) * px(f) * m.object_depth_extent_m /
                         (p.camera.focal_px * p.camera.baseline_m);
        const double so = std::sqrt(m.sigma_disp * m.sigma_disp + e * e);
        const double mass = gauss_cdf((dr - px(f)) / so) - gauss_cdf(-px(f) / so);
        h->obj_k[2 * f] = std::log(mass) + std::log(so * std::sqrt(2.0 * M_PI)) -
                          std::log(1.0 - m.p_out);
        h->obj_k[2 * f + 1] = 2.0 * so * so;
        for (int d = 0; d < D; ++d)
            h->object_t[(size_t)f * D + d] = keep(to_grid(pixel_cost(px(d), px(f), so, m.p_out, dr), g));
    }
    h->object_df.resize((size_t)D * D);
    for (int f = 0; f < D; ++f)
        for (int d = 0; d < D; ++d) h->object_df[(size_t)d * D + f] = h->object_t[(size_t)f * D + d];
    // priors
    const double beta = to_grid(m.bic_cost, g);
    double fmaxp = 0.0, tmaxp = 0.0;
    for (int a = 0; a < 3; ++a) {
        const double f = to_grid(m.first_cost[a], g) + beta;
        h->prior.first[a] = (float)f;
        fmaxp = std::fmax(fmaxp, f);
        for (int b = 0; b < 3; ++b) {
            const double t = to_grid(m.trans_cost[a][b], g) + beta;
            h->prior.trans[a][b] = (float)t;
            if (std::isfinite(t)) tmaxp = std::fmax(tmaxp, t);
        }
    }
    h->prior.c_ord = (float)to_grid(m.ordering_cost, g);
    h->prior.c_grav = (float)to_grid(m.gravity_cost, g);
    h->prior.c_dive = (float)to_grid(m.diving_cost, g);
    h->prior.tau_ord = m.ordering_tol_px << k;     // in bins
    h->prior.mean_eps = (float)std::ldexp((double)D, -22);
    h->prior.exact = g >= 0 ? 1 : 0;
    if (g < 0) {
        // costs off the grid: FP32 sums are not exact, so there is no range
        // to keep; every pose is admitted
        h->pose_in_range = true;
        return STIXELS_OK;
    }
    // exactness: every prefix, cost and intermediate of the recurrence is a
    // multiple of 2^-g bounded by 2 (h+1) cmax plus the priors
    const double bound = 2.0 * (Hmax + 1) * cmax + fmaxp + tmaxp + h->prior.c_ord +
                         h->prior.c_grav + h->prior.c_dive;
    // a frame pose (stixels_compute_pose) keeps every ground model disparity
    // in [0, d_range]; its ground costs then lie between the object cost of
    // pixel 0 at mean 0 (the smallest Gaussian cost any such model reaches)
    // and the outlier cost
    const double c_out = std::log(dr) - std::log(m.p_out);
    const double pose_bound = 2.0 * (Hmax + 1) * std::fmax(cmax, c_out) + fmaxp + tmaxp +
                              h->prior.c_ord + h->prior.c_grav + h->prior.c_dive;
    h->pose_in_range = pose_bound < std::ldexp(1.0, 24 - g);
    if (!(bound < std::ldexp(1.0, 24 - g))) {
        char buf[200];
        snprintf(buf, sizeof buf,
                 "cost range %.1f reaches 2^(24-g) = %.0f: FP32 would not be exact on the grid",
                 bound, std::ldexp(1.0, 24 - g));
        return fail(h, STIXELS_E_RANGE, buf);
    }
    return STIXELS_OK;
}

thread_local std::string g_create_error;

// Path of stixels_compute: the request, or automatically the staged kernels.
int frame_path_of(const stixels_handle* h) { return h->frame_path == 0 ? 1 : h->frame_path; }

}  // namespace

extern "C" {

int stixels_create(const stixels_params* params, stixels_handle** out) {
    if (!params || !out) return STIXELS_E_INVALID_ARG;
    *out = nullptr;
    std::string why;
    int rc = validate(params, why);
    if (rc != STIXELS_OK) {
        g_create_error = why;
        return rc;
    }
    stixels_handle* h = new (std::nothrow) stixels_handle;
    if (!h) return STIXELS_E_NOMEM;
    h->p = *params;
    h->D = params->max_disparity << params->subpixel_log2;   // disparity bins
    h->Hmax = params->max_height;
    h->Wmax = params->max_width;
    h->s = params->stixel_width;
    h->ncols_max = h->Wmax / h->s;
    rc = build_tables(h);
    if (rc == STIXELS_OK && hipGetDevice(&h->device) != hipSuccess)
        rc = fail(h, STIXELS_E_HIP, "no HIP device");
    // the fixed workspace of stixels_compute_noalloc on this device (once per
    // device; that entry point reports a failure here when it is called)
    if (rc == STIXELS_OK) (void)noalloc_setup(h->device);
    if (rc == STIXELS_OK &&
        hipDeviceGetAttribute(&h->num_cu, hipDeviceAttributeMultiprocessorCount, h->device) !=
            hipSuccess)
        rc = fail(h, STIXELS_E_HIP, "cannot read the compute unit count");
    if (rc == STIXELS_OK &&
        hipDeviceGetAttribute(&h->lds_per_block, hipDeviceAttributeMaxSharedMemoryPerBlock,
                              h->device) != hipSuccess)
        rc = fail(h, STIXELS_E_HIP, "cannot read the LDS size");
    if (rc == STIXELS_OK) rc = upload(h, &h->d_sky, h->sky);
    if (rc == STIXELS_OK) rc = upload(h, &h->d_ground, h->ground);
    if (rc == STIXELS_OK) rc = upload(h, &h->d_object_t, h->object_t);
    if (rc == STIXELS_OK) rc = upload(h, &h->d_object_df, h->object_df);
    if (rc == STIXELS_OK) rc = upload(h, &h->d_fg_hi, h->fg_hi);
    if (rc == STIXELS_OK) rc = upload(h, &h->d_fg_lo, h->fg_lo);
    if (rc == STIXELS_OK) rc = upload(h, &h->d_obj_k, h->obj_k);
    if (rc == STIXELS_OK && !(params->flags & STIXELS_FLAG_BATCH_ONLY)) {
        const size_t nc = (size_t)h->ncols_max, H1 = (size_t)h->Hmax + 1;
        // d_po holds the staged path's object prefix tables or, for the
        // fused path, its descriptor, task list and one scratch slot per
        // column
        h->ws_bytes = std::max(nc * h->D * H1 * sizeof(float) + kTableGuardBytes,
                               persist::frame_fused_bytes(h->ncols_max, h->Hmax, h->D, h->ncols_max));
        bool ok = hipMalloc(reinterpret_cast<void**>(&h->d_q), nc * h->Hmax * sizeof(int16_t)) == hipSuccess &&
                  hipMalloc(reinterpret_cast<void**>(&h->d_prefix), 4 * nc * H1 * sizeof(float)) == hipSuccess &&
                  hipMalloc(reinterpret_cast<void**>(&h->d_range), 2 * nc * sizeof(int32_t)) == hipSuccess &&
                  hipMalloc(reinterpret_cast<void**>(&h->d_po), h->ws_bytes) == hipSuccess &&
                  hipMalloc(reinterpret_cast<void**>(&h->d_pose_ground),
                            (size_t)h->Hmax * h->D * sizeof(float)) == hipSuccess &&
                  hipMalloc(reinterpret_cast<void**>(&h->d_pose_hi), (size_t)h->Hmax * sizeof(int32_t)) == hipSuccess &&
                  hipMalloc(reinterpret_cast<void**>(&h->d_pose_lo), (size_t)h->Hmax * sizeof(int32_t)) == hipSuccess;
        if (!ok) rc = fail(h, STIXELS_E_NOMEM, "hipMalloc of the frame workspace failed");
    }
    if (rc != STIXELS_OK) {
        g_create_error = h->err;
        release(h);
        delete h;
        return rc;
    }
    *out = h;
    return STIXELS_OK;
}

int stixels_destroy(stixels_handle* h) {
    if (!h) return STIXELS_OK;
    stixels_batch_destroy(h->auto_batch);
    release(h);
    delete h;
    return STIXELS_OK;
}

int stixels_device_bytes(const stixels_handle* h, size_t* bytes) {
    if (!h || !bytes) return STIXELS_E_INVALID_ARG;
    size_t n = (h->sky.size() + h->ground.size() + h->object_t.size() + h->object_df.size() +
                h->fg_hi.size() + h->fg_lo.size()) * 4;
    if (h->d_po) {
        const size_t nc = (size_t)h->ncols_max, H1 = (size_t)h->Hmax + 1;
        n += nc * h->Hmax * sizeof(int16_t) + 4 * nc * H1 * sizeof(float) +
             2 * nc * sizeof(int32_t) + h->ws_bytes +
             (size_t)h->Hmax * (h->D * sizeof(float) + 2 * sizeof(int32_t));
    }
    size_t b = 0;
    if (h->auto_batch && stixels_batch_device_bytes(h->auto_batch, &b) == STIXELS_OK) n += b;
    *bytes = n;
    return STIXELS_OK;
}

int stixels_num_columns(const stixels_handle* h, int32_t width, int32_t* ncols) {
    if (!h || !ncols || width < h->s) return STIXELS_E_INVALID_ARG;
    *ncols = width / h->s;
    return STIXELS_OK;
}

int stixels_output_capacity(const stixels_handle* h, int32_t height, int32_t* capacity) {
    if (!h || !capacity || height < 1) return STIXELS_E_INVALID_ARG;
    *capacity = h->p.max_stixels_per_column > 0 ? h->p.max_stixels_per_column : height;
    return STIXELS_OK;
}

}  // extern "C"

namespace {

// A frame through the path of stixels_compute, with the handle's camera
// (pose == nullptr) or with the frame's own pose, whose ground table is built
// on the device first.
int compute_frame(stixels_handle* h, const float* d_disparity, int32_t width, int32_t height,
                  const stixels_pose* pose, void* stream, const stixels_output* out) {
    if (!h) return STIXELS_E_INVALID_ARG;
    if (!d_disparity || !out || !out->counts || !out->records || !out->total_cost ||
        !out->overflow)
        return fail(h, STIXELS_E_INVALID_ARG, "null input or output pointer");
    if (width < h->s || width > h->Wmax)
        return fail(h, STIXELS_E_INVALID_ARG, "width outside [stixel_width, max_width]");
    if (height < 1 || height > h->Hmax)
        return fail(h, STIXELS_E_INVALID_ARG, "height outside [1, max_height]");
    if (out->capacity < 1) return fail(h, STIXELS_E_INVALID_ARG, "output capacity must be >= 1");
    if (!h->d_po)
        return fail(h, STIXELS_E_INVALID_ARG, "handle created for the batch API only (no workspace)");
    const hipStream_t st = static_cast<hipStream_t>(stream);
    DeviceModel m = device_model(h);
    // costs off the grid run the fused kernel with stored links
    const int path = h->prior.exact ? frame_path_of(h) : 2;
    if (pose) {
        if (!h->pose_in_range)
            return fail(h, STIXELS_E_RANGE,
                        "the handle's cost range leaves no room for frame poses (exact grid)");
        PoseItem it{};
        const char* why = "";
        const int rc = make_pose_item(h->p, h->D, *pose, height, h->d_pose_ground, h->d_pose_hi,
                                      h->d_pose_lo, &it, &why);
        if (rc != STIXELS_OK) return fail(h, rc, why);
        const hipError_t e = launch_pose_tables(it, st);
        if (e != hipSuccess)
            return fail(h, STIXELS_E_HIP, std::string("pose table launch failed: ") + hipGetErrorString(e));
        m.ground = h->d_pose_ground;
        m.fg_hi = h->d_pose_hi;
        m.fg_lo = h->d_pose_lo;
        m.horizon_row = pose->horizon_row;
    }
    const int waves = frame_waves(h->waves, height, width / h->s, h->num_cu);
    if (path == 2) {
        int grid = 0;
        persist::JobDesc job = persist::make_job_desc(h, d_disparity, width, height, *out);
        job.ground = m.ground;
        job.fg_hi = m.fg_hi;
        job.fg_lo = m.fg_lo;
        job.vtop = ground_top(m.horizon_row, height);
        const hipError_t e = persist::launch_frame_fused(job, h->d_po, h->ws_bytes, waves,
                                                         h->num_cu, st, &grid);
        if (e != hipSuccess)
            return fail(h, STIXELS_E_HIP, std::string("kernel launch failed: ") + hipGetErrorString(e));
        h->last_W = width;
        h->last_H = height;
        h->last_path = 2;
        return STIXELS_OK;
    }
    const int ncols = width / h->s;
    const int vtop = ground_top(m.horizon_row, height);
    FrameWorkspace ws{h->d_q, h->d_prefix, h->d_range, h->d_po};
    FrameOutput fo{out->counts, reinterpret_cast<uint32_t*>(out->records), out->total_cost,
                   out->overflow, out->capacity};
    hipError_t e = launch_reduce(m, d_disparity, width, height, ncols, ws.q, st);
    if (e == hipSuccess) e = launch_tables(m, ws, height, ncols, vtop, st);
    if (e == hipSuccess)
        e = launch_dp(m, ws, height, ncols, vtop, waves, frame_po_lds(h->po_placement, height),
                      h->lds_per_block, fo, st);
    if (e != hipSuccess)
        return fail(h, STIXELS_E_HIP, std::string("kernel launch failed: ") + hipGetErrorString(e));
    h->last_W = width;
    h->last_H = height;
    h->last_path = 1;
    return STIXELS_OK;
}

}  // namespace

extern "C" {

int stixels_compute(stixels_handle* h, const float* d_disparity, int32_t width, int32_t height,
                    void* stream, const stixels_output* out) {
    return compute_frame(h, d_disparity, width, height, nullptr, stream, out);
}

int stixels_compute_pose(stixels_handle* h, const float* d_disparity, int32_t width,
                         int32_t height, const stixels_pose* pose, void* stream,
                         const stixels_output* out) {
    if (!h) return STIXELS_E_INVALID_ARG;
    if (!pose) return fail(h, STIXELS_E_INVALID_ARG, "null pose");
    return compute_frame(h, d_disparity, width, height, pose, stream, out);
}

int stixels_debug_pose_tables(stixels_handle* h, const stixels_pose* pose, int32_t height,
                              void* host_dst, size_t bytes, void* stream) {
    if (!h) return STIXELS_E_INVALID_ARG;
    if (!pose || !host_dst || height < 1 || height > h->Hmax || !h->d_pose_ground)
        return fail(h, STIXELS_E_INVALID_ARG, "null pose or buffer, height out of range or batch-only handle");
    const size_t gbytes = (size_t)height * h->D * sizeof(float);
    const size_t tbytes = (size_t)height * sizeof(int32_t);
    if (bytes != gbytes + 2 * tbytes)
        return fail(h, STIXELS_E_INVALID_ARG, "bytes must equal height * (4 d_range + 8)");
    PoseItem it{};
    const char* why = "";
    const int rc = make_pose_item(h->p, h->D, *pose, height, h->d_pose_ground, h->d_pose_hi,
                                  h->d_pose_lo, &it, &why);
    if (rc != STIXELS_OK) return fail(h, rc, why);
    const hipStream_t st = static_cast<hipStream_t>(stream);
    char* dst = static_cast<char*>(host_dst);
    hipError_t e = launch_pose_tables(it, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e == hipSuccess) e = hipMemcpy(dst, h->d_pose_ground, gbytes, hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemcpy(dst + gbytes, h->d_pose_hi, tbytes, hipMemcpyDeviceToHost);
    if (e == hipSuccess)
        e = hipMemcpy(dst + gbytes + tbytes, h->d_pose_lo, tbytes, hipMemcpyDeviceToHost);
    if (e != hipSuccess)
        return fail(h, STIXELS_E_HIP, std::string("pose tables failed: ") + hipGetErrorString(e));
    return STIXELS_OK;
}

int stixels_debug_stage_times(stixels_handle* h, const float* d_disparity, int32_t width,
                              int32_t height, void* stream, const stixels_output* out,
                              float* host_ms) {
    if (!h || !host_ms) return STIXELS_E_INVALID_ARG;
    if (!d_disparity || !out || !out->counts || !out->records || !out->total_cost ||
        !out->overflow || out->capacity < 1 || width < h->s || width > h->Wmax || height < 1 ||
        height > h->Hmax || !h->d_po)
        return fail(h, STIXELS_E_INVALID_ARG, "invalid frame, output or batch-only handle");
    if (!h->prior.exact)
        return fail(h, STIXELS_E_INVALID_ARG, "costs off the grid run the fused path only");
    const hipStream_t st = static_cast<hipStream_t>(stream);
    const int ncols = width / h->s;
    const int vtop = ground_top(h->p.camera.horizon_row, height);
    const int waves = frame_waves(h->waves, height, ncols, h->num_cu);
    DeviceModel m = device_model(h);
    FrameWorkspace ws{h->d_q, h->d_prefix, h->d_range, h->d_po};
    FrameOutput fo{out->counts, reinterpret_cast<uint32_t*>(out->records), out->total_cost,
                   out->overflow, out->capacity};
    hipEvent_t ev[4] = {};
    hipError_t e = hipSuccess;
    for (int i = 0; i < 4 && e == hipSuccess; ++i) e = hipEventCreate(&ev[i]);
    if (e == hipSuccess) e = hipEventRecord(ev[0], st);
    if (e == hipSuccess) e = launch_reduce(m, d_disparity, width, height, ncols, ws.q, st);
    if (e == hipSuccess) e = hipEventRecord(ev[1], st);
    if (e == hipSuccess) e = launch_tables(m, ws, height, ncols, vtop, st);
    if (e == hipSuccess) e = hipEventRecord(ev[2], st);
    if (e == hipSuccess)
        e = launch_dp(m, ws, height, ncols, vtop, waves, frame_po_lds(h->po_placement, height),
                      h->lds_per_block, fo, st);
    if (e == hipSuccess) e = hipEventRecord(ev[3], st);
    if (e == hipSuccess) e = hipEventSynchronize(ev[3]);
    for (int i = 0; i < 3 && e == hipSuccess; ++i) e = hipEventElapsedTime(&host_ms[i], ev[i], ev[i + 1]);
    for (int i = 0; i < 4; ++i)
        if (ev[i]) (void)hipEventDestroy(ev[i]);
    if (e != hipSuccess)
        return fail(h, STIXELS_E_HIP, std::string("timed staged frame failed: ") + hipGetErrorString(e));
    h->last_W = width;
    h->last_H = height;
    h->last_path = 1;
    return STIXELS_OK;
}

int stixels_set_frame_path(stixels_handle* h, int32_t path) {
    if (!h) return STIXELS_E_INVALID_ARG;
    if (path < 0 || path > 2)
        return fail(h, STIXELS_E_INVALID_ARG, "frame path must be 0 (auto), 1 (staged) or 2 (fused)");
    h->frame_path = path;
    return STIXELS_OK;
}

int stixels_set_object_lut(stixels_handle* h, int32_t mode) {
    if (!h) return STIXELS_E_INVALID_ARG;
    if (mode != 0 && mode != 1)
        return fail(h, STIXELS_E_INVALID_ARG, "object LUT mode must be 0 (offline) or 1 (online)");
    h->object_lut = mode;
    return STIXELS_OK;
}

int stixels_get_frame_path(const stixels_handle* h) {
    return h ? (h->prior.exact ? frame_path_of(h) : 2) : 0;
}

int stixels_output_bytes(const stixels_handle* h, int32_t width, int32_t height, size_t* bytes) {
    int32_t ncols = 0, cap = 0;
    if (!bytes || stixels_num_columns(h, width, &ncols) != STIXELS_OK ||
        stixels_output_capacity(h, height, &cap) != STIXELS_OK)
        return STIXELS_E_INVALID_ARG;
    *bytes = (size_t)ncols * (sizeof(int32_t) + (size_t)cap * sizeof(stixels_record) +
                              sizeof(float) + sizeof(uint8_t));
    return STIXELS_OK;
}

int stixels_set_waves(stixels_handle* h, int32_t waves) {
    if (!h) return STIXELS_E_INVALID_ARG;
    if (waves != 0 && waves != 1 && waves != 2 && waves != 4)
        return fail(h, STIXELS_E_INVALID_ARG, "waves per column must be 0, 1, 2 or 4");
    h->waves = waves;
    return STIXELS_OK;
}

int stixels_set_po_placement(stixels_handle* h, int32_t placement) {
    if (!h) return STIXELS_E_INVALID_ARG;
    if (placement < 0 || placement > 2)
        return fail(h, STIXELS_E_INVALID_ARG, "placement must be 0 (auto), 1 (HBM) or 2 (LDS)");
    h->po_placement = placement;
    return STIXELS_OK;
}

int stixels_get_waves(const stixels_handle* h, int32_t height, int32_t width) {
    if (!h || height < 1 || width < h->s) return 0;
    return frame_waves(h->waves, height, width / h->s, h->num_cu);
}

const char* stixels_last_error(const stixels_handle* h) {
    if (!h) return g_create_error.c_str();
    return h->err.c_str();
}

const char* stixels_status_string(int code) {
    switch (code) {
        case STIXELS_OK: return "ok";
        case STIXELS_E_INVALID_ARG: return "invalid argument";
        case STIXELS_E_RANGE: return "parameters outside the exact cost range";
        case STIXELS_E_HIP: return "HIP error";
        case STIXELS_E_NOMEM: return "out of memory";
        default: return "unknown status";
    }
}

namespace {
int copy_table(const stixels_handle* h, int32_t which, void* host_dst, size_t bytes) {
    const void* src = nullptr;
    size_t n = 0;
    switch (which) {
        case STIXELS_TABLE_SKY: src = h->sky.data(); n = h->sky.size() * 4; break;
        case STIXELS_TABLE_GROUND: src = h->ground.data(); n = h->ground.size() * 4; break;
        case STIXELS_TABLE_OBJECT: src = h->object_t.data(); n = h->object_t.size() * 4; break;
        case STIXELS_TABLE_FG_HI: src = h->fg_hi.data(); n = h->fg_hi.size() * 4; break;
        case STIXELS_TABLE_FG_LO: src = h->fg_lo.data(); n = h->fg_lo.size() * 4; break;
        default: return STIXELS_E_INVALID_ARG;
    }
    if (bytes != n) return STIXELS_E_INVALID_ARG;
    std::memcpy(host_dst, src, n);
    return STIXELS_OK;
}
}  // namespace

int stixels_debug_table(const stixels_handle* h, int32_t which, void* host_dst, size_t bytes) {
    if (!h || !host_dst) return STIXELS_E_INVALID_ARG;
    return copy_table(h, which, host_dst, bytes);
}

int stixels_debug_tables(const stixels_handle* h, void* host_dst, size_t bytes) {
    if (!h || !host_dst) return STIXELS_E_INVALID_ARG;
    const size_t parts[5] = {h->sky.size() * 4, h->ground.size() * 4, h->object_t.size() * 4,
                             h->fg_hi.size() * 4, h->fg_lo.size() * 4};
    size_t total = 0;
    for (size_t x : parts) total += x;
    if (bytes != total) return STIXELS_E_INVALID_ARG;
    char* dst = static_cast<char*>(host_dst);
    for (int which = 0; which < 5; ++which) {
        const int rc = copy_table(h, which, dst, parts[which]);
        if (rc != STIXELS_OK) return rc;
        dst += parts[which];
    }
    return STIXELS_OK;
}

int stixels_host_table(const stixels_params* params, int32_t which, void* host_dst,
                       size_t bytes) {
    if (!params || !host_dst) return STIXELS_E_INVALID_ARG;
    std::string why;
    int rc = validate(params, why);
    if (rc != STIXELS_OK) {
        g_create_error = why;
        return rc;
    }
    stixels_handle h;
    h.p = *params;
    h.D = params->max_disparity << params->subpixel_log2;
    h.Hmax = params->max_height;
    h.Wmax = params->max_width;
    h.s = params->stixel_width;
    rc = build_tables(&h);
    if (rc != STIXELS_OK) {
        g_create_error = h.err;
        return rc;
    }
    return copy_table(&h, which, host_dst, bytes);
}

int stixels_debug_stage(const stixels_handle* h, int32_t which, void* host_dst, size_t bytes,
                        void* stream) {
    if (!h || !host_dst || h->last_H < 1) return STIXELS_E_INVALID_ARG;
    if (h->last_path != 1) return STIXELS_E_INVALID_ARG;   // the fused path keeps no per-frame tables
    const size_t ncols = (size_t)(h->last_W / h->s), H = (size_t)h->last_H;
    const void* src = nullptr;
    size_t n = 0;
    switch (which) {
        case STIXELS_STAGE_REDUCED: src = h->d_q; n = ncols * H * 2; break;
        case STIXELS_STAGE_PREFIX: src = h->d_prefix; n = 4 * ncols * (H + 1) * 4; break;
        case STIXELS_STAGE_RANGE: src = h->d_range; n = 2 * ncols * 4; break;
        case STIXELS_STAGE_OBJECT_PREFIX: src = h->d_po; n = ncols * h->D * (H + 1) * 4; break;
        default: return STIXELS_E_INVALID_ARG;
    }
    if (bytes != n) return STIXELS_E_INVALID_ARG;
    if (hipStreamSynchronize(static_cast<hipStream_t>(stream)) != hipSuccess) return STIXELS_E_HIP;
    if (hipMemcpy(host_dst, src, n, hipMemcpyDeviceToHost) != hipSuccess) return STIXELS_E_HIP;
    return STIXELS_OK;
}

int stixels_selftest_mean(int32_t d_range, int32_t max_height, int64_t* host_mismatches) {
    if (!host_mismatches || d_range < 2 || d_range > kMaxDisparity || max_height < 1 ||
        max_height > kMaxHeight || (long long)max_height * d_range > (1LL << 20))
        return STIXELS_E_INVALID_ARG;
    return run_selftest_mean(d_range, max_height, host_mismatches) == hipSuccess ? STIXELS_OK
                                                                                  : STIXELS_E_HIP;
}

}  // extern "C"
