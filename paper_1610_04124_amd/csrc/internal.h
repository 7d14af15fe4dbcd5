// internal.h -- device building blocks of the gfx950 stixel library.
//
// Layout in HBM (per frame, per reduced column i of height h):
//   q      int16 [ncols][h]            reduced disparities, bottom-up, -1 invalid
//   prefix float [4][ncols][h+1]       PG (ground), PS (sky), PA = 2*sum(q)+count,
//                                      PN2 = 2*count; entry v+1 covers rows 0..v
//   range  int32 [ncols][2]            smallest / largest valid q of the column
//   PO     float [ncols][D][h+1]       object prefix table, row f-fmin holds
//                                      sum over rows of O[q_v][f]
// Every cost value is a multiple of 2^-g and every partial sum stays below
// 2^(24-g) in magnitude (checked when a handle is created), so FP32 adds,
// subtractions and minima are exact and their order does not matter.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "stixels.h"

namespace stx {

constexpr int kWave = 64;
constexpr int kMaxSlots = 16;          // rows per lane in the recurrence: h <= 1024
constexpr int kMaxHeight = kWave * kMaxSlots;
constexpr int kMaxStixelWidth = 16;
constexpr int kMaxDisparity = 256;
constexpr uint32_t kBufferWord3 = 0x00020000u;  // raw buffer resource, gfx9 family
// Bytes allocated past the end of every object prefix table workspace: the
// recurrence's gathers for rows past a column's height may read up to 64 S
// floats beyond the column's last table row (their values are never used),
// and this keeps those reads inside the allocation.
constexpr size_t kTableGuardBytes = 64 * 1024;

// Instantiated slot counts of the recurrence kernels (64-row slots per lane);
// a column runs on the smallest one that covers its height.
__host__ __device__ constexpr int kernel_slots(int h) {
    const int s = (h + 63) / 64;
    return s <= 8 ? s : (s <= 10 ? 10 : (s <= 12 ? 12 : (s <= 14 ? 14 : 16)));
}
// 64-entry disparity chunks for a d_range.
__host__ __device__ constexpr int kernel_chunks(int d_range) { return d_range <= 128 ? 2 : 4; }

// Instantiated (slots, disparity chunks, waves per column) triples.
#define STX_FOR_EACH_VARIANT(X) \
    X(1, 2, 1) X(2, 2, 1) X(2, 2, 2) X(3, 2, 1) X(3, 2, 2) X(4, 2, 1) X(4, 2, 2) X(4, 2, 4) \
    X(5, 2, 1) X(5, 2, 2) X(5, 2, 4) X(6, 2, 1) X(6, 2, 2) X(6, 2, 4) X(7, 2, 1) X(7, 2, 2) \
    X(7, 2, 4) X(8, 2, 1) X(8, 2, 2) X(8, 2, 4) X(10, 2, 1) X(10, 2, 2) X(10, 2, 4) \
    X(12, 2, 1) X(12, 2, 2) X(12, 2, 4) X(14, 2, 1) X(14, 2, 2) X(14, 2, 4) X(16, 2, 1) \
    X(16, 2, 2) X(16, 2, 4) X(1, 4, 1) X(2, 4, 1) X(2, 4, 2) X(3, 4, 1) X(3, 4, 2) \
    X(4, 4, 1) X(4, 4, 2) X(4, 4, 4) X(5, 4, 1) X(5, 4, 2) X(5, 4, 4) X(6, 4, 1) X(6, 4, 2) \
    X(6, 4, 4) X(7, 4, 1) X(7, 4, 2) X(7, 4, 4) X(8, 4, 1) X(8, 4, 2) X(8, 4, 4) X(10, 4, 1) \
    X(10, 4, 2) X(10, 4, 4) X(12, 4, 1) X(12, 4, 2) X(12, 4, 4) X(14, 4, 1) X(14, 4, 2) \
    X(14, 4, 4) X(16, 4, 1) X(16, 4, 2) X(16, 4, 4)

// Variants of the recurrence that keep an index table of cut positions
// (Sec. 3.3) for the backtracking, used by handles whose costs are not on a
// grid (cost_grid_log2 = -1): one wave per column, every slot count and
// disparity chunk count.
#define STX_FOR_EACH_LINKS_VARIANT(X) \
    X(1, 2) X(2, 2) X(3, 2) X(4, 2) X(5, 2) X(6, 2) X(7, 2) X(8, 2) X(10, 2) X(12, 2) \
    X(14, 2) X(16, 2) X(1, 4) X(2, 4) X(3, 4) X(4, 4) X(5, 4) X(6, 4) X(7, 4) X(8, 4) \
    X(10, 4) X(12, 4) X(14, 4) X(16, 4)

// Slot counts of the two-columns-per-wave recurrence (d_range <= 128, h <= 512).
#define STX_FOR_EACH_PAIR_VARIANT(X) \
    X(1, 2) X(2, 2) X(3, 2) X(4, 2) X(5, 2) X(6, 2) X(7, 2) X(8, 2)

// Quantised prior constants of one camera model, in FP32 (exact on the grid).
struct Prior {
    float first[3];       // F[c] + beta
    float trans[3][3];    // T[prev][cur] + beta (INFINITY when forbidden)
    float c_ord, c_grav, c_dive;
    int tau_ord;
    float mean_eps;       // bias of the rounded-mean division, d_range * 2^-22
    int exact;            // 1: every cost is on the 2^-g grid (FP32 sums are exact)
};

// Per-frame geometry shared by the kernels.
struct FrameGeom {
    int W, H, s, ncols, D;
    int vtop;             // highest bottom-up row a ground stixel may reach
    int reduce_mode;
    int sub;              // disparity bins of 2^-sub px
};

__device__ __forceinline__ float inf_f() { return __builtin_inff(); }

__device__ __forceinline__ float readlane_f(float v, int lane) {
    return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), lane));
}
__device__ __forceinline__ int readlane_i(int v, int lane) {
    return __builtin_amdgcn_readlane(v, lane);
}
// v with lane `lane` replaced by the wave-uniform value x.
__device__ __forceinline__ float writelane_f(float x, int lane, float v) {
    return ((int)(threadIdx.x & 63) == lane) ? x : v;
}

// ------------------------------------------------------------------ Sec. 4.1
// One reduced pixel from the s disparities of a row strip: lower median (mode
// 0) or FP64 mean (mode 1) of the valid values, in bins of 2^-sub px
// (scaled by 2^sub, exact), rounded half to even and clamped to the last
// bin D-1; -1 when no value is valid.  The median is an exact rank
// selection: the value whose rank (ties broken by position) is (n-1)/2.
template <int S>
__device__ __forceinline__ int reduce_strip(const float* __restrict__ p, int mode, int D,
                                            int sub) {
    float x[S];
    bool ok[S];
    int n = 0;
#pragma unroll
    for (int t = 0; t < S; ++t) {
        x[t] = p[t];
        ok[t] = (x[t] >= 0.0f) && (x[t] <= 3.402823466e38f);
        n += ok[t] ? 1 : 0;
    }
    if (n == 0) return -1;
    if (mode == 0) {
        const int want = (n - 1) >> 1;
        float med = 0.0f;
#pragma unroll
        for (int i = 0; i < S; ++i) {
            int rank = 0;
#pragma unroll
            for (int j = 0; j < S; ++j) {
                const bool before = (x[j] < x[i]) || (x[j] == x[i] && j < i);
                rank += (ok[j] && before) ? 1 : 0;
            }
            if (ok[i] && rank == want) med = x[i];
        }
        const float r = __builtin_rintf(__builtin_ldexpf(med, sub));
        const float top = (float)(D - 1);
        return (int)(r < top ? r : top);
    }
    double sum = 0.0;
#pragma unroll
    for (int t = 0; t < S; ++t)
        if (ok[t]) sum += (double)x[t];
    const double r = __builtin_rint(__builtin_ldexp(sum / (double)n, sub));
    const double top = (double)(D - 1);
    return (int)(r < top ? r : top);
}

// ------------------------------------------------------------------ scans
// Inclusive prefix sum over the 64 lanes of a wave with DPP row shifts and
// row broadcasts (exact: every addend is on the cost grid or an integer).
template <int CTRL, int ROWMASK>
__device__ __forceinline__ float dpp_shift(float x) {
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, x),
                                                                 CTRL, ROWMASK, 0xf, true));
}

__device__ __forceinline__ float wave_inclusive_scan(float x) {
    x += dpp_shift<0x111, 0xf>(x);   // row_shr:1
    x += dpp_shift<0x112, 0xf>(x);   // row_shr:2
    x += dpp_shift<0x114, 0xf>(x);   // row_shr:4
    x += dpp_shift<0x118, 0xf>(x);   // row_shr:8
    x += dpp_shift<0x142, 0xa>(x);   // row_bcast:15 into rows 1 and 3
    x += dpp_shift<0x143, 0xc>(x);   // row_bcast:31 into rows 2 and 3
    return x;
}

// IEEE 754-2019 minimum: a single v_minimum3_f32 on gfx950, with no
// operand canonicalisation (fminf adds one per operand).  The two agree on
// every value the recurrence produces: no NaN, and no -0.
__device__ __forceinline__ float vmin(float a, float b) {
    return __builtin_elementwise_minimum(a, b);
}

// ------------------------------------------------------------------ Sec. 3.4
// Rounded mean of a stixel's valid disparities, floor((2S+n)/(2n)), minus a
// caller-chosen integer base <= the mean, from the prefix differences
// a = 2S+n and n2 = 2n (both exact integers in FP32); c = eps - base with
// eps = d_range * 2^-22.  With r = rcp(n2) (relative error <= 2^-23),
// fma(a, r, eps) lies in [m, m+1) whenever a / n2 lies in [m, m+1) and
// 2n * d_range < 2^24 / 7, which handle creation enforces (h * d_range <=
// 2^20); shifting by the integer base keeps the exact value the same
// distance from the integers and cannot enlarge the rounding error, so the
// truncation gives m - base.  n = 0 (a = 0): rcp gives +inf, the product
// NaN, and v_cvt_i32_f32 turns NaN into 0; callers use base 0 whenever a
// stixel without valid pixels can occur.  stixels_selftest_mean checks all
// of this on the device.
__device__ __forceinline__ int cvt_i32_nan0(float x) {
    int r;
    asm("v_cvt_i32_f32 %0, %1" : "=v"(r) : "v"(x));
    return r;
}
__device__ __forceinline__ int mean_index(float a, float n2, float c) {
    return cvt_i32_nan0(__builtin_fmaf(a, __builtin_amdgcn_rcpf(n2), c));
}
__device__ __forceinline__ int rounded_mean(float a, float n2, float eps) {
    return mean_index(a, n2, eps);
}

__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void* base, uint32_t bytes) {
    // base and bytes are the same in every lane; reading them from the first
    // lane lets the compiler keep the resource in scalar registers (otherwise
    // each load through it is wrapped in a loop over distinct lane values)
    const uint64_t p = reinterpret_cast<uint64_t>(base);
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)p);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(p >> 32));
    void* ub = reinterpret_cast<void*>(((uint64_t)hi << 32) | lo);
    return __builtin_amdgcn_make_buffer_rsrc(ub, (short)0, (int)__builtin_amdgcn_readfirstlane(bytes),
                                             (int)kBufferWord3);
}

// Load element `idx` (float) through a bounds-checked buffer resource: an
// index past the resource's size reads 0 instead of faulting.
__device__ __forceinline__ float buf_load(__amdgpu_buffer_rsrc_t r, int idx) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, idx * 4, 0, 0));
}

// Same with a per-lane byte offset and a wave-uniform byte offset (SGPR).
__device__ __forceinline__ float buf_load_b(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
    return __builtin_bit_cast(float,
                              __builtin_amdgcn_raw_buffer_load_b32(r, (int)voff, (int)soff, 0));
}

// Store a float through a buffer resource at a per-lane byte offset plus a
// wave-uniform byte offset (SGPR).  A vector-memory store; an offset past
// the resource's size is dropped.
__device__ __forceinline__ void buf_store_b(__amdgpu_buffer_rsrc_t r, float x, uint32_t voff,
                                            uint32_t soff) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, x), r, (int)voff, (int)soff,
                                          0);
}

// Four consecutive floats with one 16-byte store (voff + soff 16-byte aligned).
__device__ __forceinline__ void buf_store_b4(__amdgpu_buffer_rsrc_t r, float x0, float x1, float x2,
                                             float x3, uint32_t voff, uint32_t soff) {
    typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
    const u32x4 v = {__builtin_bit_cast(uint32_t, x0), __builtin_bit_cast(uint32_t, x1),
                     __builtin_bit_cast(uint32_t, x2), __builtin_bit_cast(uint32_t, x3)};
    __builtin_amdgcn_raw_buffer_store_b128(v, r, (int)voff, (int)soff, 0);
}

}  // namespace stx
