// frame_kernels.hip -- the per-frame pipeline of Sec. 4 as three gfx950 kernels:
//   reduce  (Sec. 4.1)  s-pixel strips -> one reduced disparity, transposed to
//                       bottom-up columns through an LDS tile so that both the
//                       row-major reads and the column-major writes coalesce;
//   tables  (Sec. 4.2)  per column: ground / sky / disparity / count prefix
//                       sums and the object prefix table over the column's
//                       own disparity range, with DPP wave scans;
//   dp      (Sec. 4.3-4.4)  the recurrence and backtracking, one wave64 per
//                       column (dp_kernel.h, instantiated in inst_s*.hip).
#include <algorithm>
#include <climits>
#include <map>
#include <mutex>

#include "dp_kernel.h"
#include "kernel_table.h"
#include "launch.h"

namespace stx {

// ------------------------------------------------------------------ reduce
// One workgroup reduces a tile of 64 columns x 16 image rows (enough
// workgroups to spread one frame over the chip).
template <int S>
__global__ __launch_bounds__(256) void reduce_kernel(const float* __restrict__ disp, int W, int H,
                                                     int ncols, int D, int mode, int sub,
                                                     int16_t* __restrict__ q) {
    __shared__ int16_t tile[64][17];
    const int c0 = blockIdx.x * 64, r0 = blockIdx.y * 16;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    const int col = c0 + tx;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int rl = ty + 4 * i;
        const int r = r0 + rl;
        int v = -1;
        if (col < ncols && r < H)
            v = reduce_strip<S>(disp + (size_t)r * W + (size_t)col * S, mode, D, sub);
        tile[tx][rl] = (int16_t)v;
    }
    __syncthreads();
    // tile row rl (image row r0+rl) lands at bottom-up row H-1-r: write each
    // column's 16 rows as one contiguous run of ascending v
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int e = threadIdx.x + 256 * i;
        const int cl = e >> 4, vl = e & 15;
        const int rl = 15 - vl;
        const int r = r0 + rl;
        const int cg = c0 + cl;
        if (cg < ncols && r < H) q[(size_t)cg * H + (H - 1 - r)] = tile[cl][rl];
    }
}

// ------------------------------------------------------------------ tables
struct TablesArgs {
    const int16_t* q;
    float* prefix;
    int32_t* range;
    float* po;
    const float* sky;
    const float* ground;
    const float* object_t;
    // online object costs (instead of the offline LUT of Sec. 3.4): per mean
    // f, the Gaussian's constant part and 2 sigma^2 (FP64), the outlier cost
    const double* obj_k;
    double c_out;
    int online, g, sub;
    int H, ncols, D;
};

// Eq. 4 for pixel bin q against mean bin f, evaluated in FP64 from the
// mean's constant part k[2f] and its 2 sigma^2 k[2f+1] with the operations
// and order of the offline table build, then rounded to the grid: equal to
// the offline LUT entry bit for bit.
__device__ __forceinline__ float object_cost_online(const TablesArgs& a, int q, int f) {
    const double x = ldexp((double)q, -a.sub), mu = ldexp((double)f, -a.sub);
    const double gs = a.obj_k[2 * f] + (x - mu) * (x - mu) / a.obj_k[2 * f + 1];
    double c = a.c_out;
    if (isfinite(gs) && gs < c) c = gs;
    return (a.g >= 0) ? (float)ldexp(rint(ldexp(c, a.g)), -a.g) : (float)c;
}

__global__ __launch_bounds__(512) void tables_kernel(TablesArgs a) {
    __shared__ int16_t qs[kMaxHeight];
    __shared__ int smin, smax, sinv;
    const int col = blockIdx.x;
    const int H = a.H, D = a.D, ncols = a.ncols;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    if (tid == 0) {
        smin = INT_MAX;
        smax = -1;
        sinv = 0;
    }
    __syncthreads();
    int lmin = INT_MAX, lmax = -1, linv = 0;
    for (int v = tid; v < H; v += 512) {
        const int x = a.q[(size_t)col * H + v];
        qs[v] = (int16_t)x;
        if (x >= 0) {
            lmin = min(lmin, x);
            lmax = max(lmax, x);
        } else {
            linv = 1;
        }
    }
    atomicMin(&smin, lmin);
    atomicMax(&smax, lmax);
    atomicOr(&sinv, linv);
    __syncthreads();
    // Object means of the column's stixels lie in [smallest, largest valid
    // q]; a stixel without valid pixels has mean 0, so the table also starts
    // at 0 when the column holds an invalid pixel.
    int fmin = sinv ? 0 : smin, fmax = smax;
    if (fmax < 0) {
        fmin = 0;
        fmax = 0;
    }
    const int stride = H + 1;

    if (wave < 4) {
        // wave t scans small table t: ground, sky, 2q+1 and 2 over the valid
        // pixels (four chains side by side rather than one after another)
        const int t = __builtin_amdgcn_readfirstlane(wave);
        float* P = a.prefix + ((size_t)t * ncols + col) * stride;
        if (lane == 0) {
            P[0] = 0.0f;
            if (t == 0) {
                a.range[2 * col] = fmin;
                a.range[2 * col + 1] = fmax;
            }
        }
        float carry = 0.0f;
        for (int base = 0; base < H; base += 64) {
            const int v = base + lane;
            const int x = (v < H) ? (int)qs[v] : -1;
            float e = 0.0f;
            if (x >= 0) {
                e = (t == 0) ? a.ground[(size_t)(H - 1 - v) * D + x]
                  : (t == 1) ? a.sky[x]
                  : (t == 2) ? (float)(2 * x + 1) : 2.0f;
            }
            e = wave_inclusive_scan(e) + carry;
            if (v < H) P[v + 1] = e;
            carry = readlane_f(e, 63);
        }
    }

    // Object rows f = fmin + wave, fmin + wave + 8, ...: row f of the object
    // cost table (the cost of mean f for every pixel bin) is staged in this
    // wave's LDS by a few coalesced loads (the next row's in flight while a
    // row is scanned; a zero after it for invalid pixels and rows past H);
    // lane l takes the costs of rows 256 u + 4 l .. 256 u + 4 l + 3 from the
    // stage, sums them in order and adds the wave scan of the lanes' sums: one
    // scan per 256 rows instead of one per 64, two cost loads per row instead
    // of a gather per 64 rows.  Every cost is on the grid, so the prefixes are
    // the same bits in any order of summation.
    __shared__ float ostg[8][256 + 4];
    float* PO = a.po + (size_t)col * D * stride;
    const auto otr = make_rsrc(a.object_t, (uint32_t)(D * D) * 4u);
    const auto pow_ = make_rsrc(PO, (uint32_t)(fmax - fmin + 1) * (uint32_t)stride * 4u);
    constexpr int U = kMaxHeight / 256;          // 256-row groups
    constexpr int NC = 4;                        // 64-bin chunks of a cost row (<= 256 bins)
    const int nu = (H + 255) >> 8, nch = (D + 63) >> 6;
    float* const stg = ostg[wave];
    if (lane == 0) stg[D] = 0.0f;
    int qi[U][4];                                // stage index of each row's cost
#pragma unroll
    for (int u = 0; u < U; ++u) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int v = 256 * u + 4 * lane + i;
            const int x = (v < H) ? (int)qs[v] : -1;
            qi[u][i] = (x >= 0) ? x : D;
        }
    }
    float onext[NC];
    auto load_row = [&](int f) {
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            if (c >= nch) break;
            const int d = 64 * c + lane;
            if (a.online) {
                onext[c] = (d < D) ? object_cost_online(a, d, f) : 0.0f;
            } else {
                onext[c] = buf_load_b(otr, (uint32_t)d * 4u, (uint32_t)(f * D) * 4u);
            }
        }
    };
    const int f0 = __builtin_amdgcn_readfirstlane(fmin), f1 = __builtin_amdgcn_readfirstlane(fmax);
    if (f0 + wave <= f1) load_row(f0 + wave);
#pragma unroll 1
    for (int f = f0 + wave; f <= f1; f += 8) {
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            if (c >= nch) break;
            if (64 * c + lane < D) stg[64 * c + lane] = onext[c];
        }
        if (f + 8 <= f1) load_row(f + 8);
        const uint32_t rowoff = (uint32_t)(f - f0) * (uint32_t)stride * 4u;
        if (lane == 0) buf_store_b(pow_, 0.0f, 0u, rowoff);
        float carry = 0.0f;
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (u >= nu) break;
            const float o0 = stg[qi[u][0]], o1 = stg[qi[u][1]];
            const float o2 = stg[qi[u][2]], o3 = stg[qi[u][3]];
            const float a1 = o0 + o1, a2 = a1 + o2, a3 = a2 + o3;
            const float incl = wave_inclusive_scan(a3);
            const float e = (incl - a3) + carry;
            const float r[4] = {e + o0, e + a1, e + a2, e + a3};
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int v = 256 * u + 4 * lane + i;
                if (v < H) buf_store_b(pow_, r[i], (uint32_t)(v + 1) * 4u, rowoff);
            }
            carry = readlane_f(incl, 63) + carry;
        }
    }
}

// ------------------------------------------------------------------ self-test
__global__ __launch_bounds__(256) void selftest_mean_kernel(int D, float eps,
                                                            unsigned long long* bad) {
    // block n tests every disparity sum of n valid pixels (n = 0: the empty
    // stixel), with base 0, base = the mean and base = half the mean
    const int n = blockIdx.x;
    const long long smax = (long long)n * (D - 1);
    unsigned long long local = 0;
    for (long long S = threadIdx.x; S <= smax; S += 256) {
        const int a = (int)(2 * S + n);
        const int want = (n > 0) ? a / (2 * n) : 0;
        const int bases[3] = {0, want, want / 2};
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            const int got = mean_index((float)a, (float)(2 * n), eps - (float)bases[i]);
            local += (got != want - bases[i]) ? 1ull : 0ull;
        }
    }
    if (local) atomicAdd(bad, local);
}

// ------------------------------------------------------------------ launchers
int ground_top(double horizon_row, int H) {
    const double vh = floor((double)(H - 1) - horizon_row);
    if (vh < -1.0) return -1;
    if (vh > (double)H) return H;
    return (int)vh;
}

template <int S>
static void reduce_launch(dim3 g, const DeviceModel& m, const float* disp, int W, int H, int ncols,
                          int16_t* q, hipStream_t st) {
    hipLaunchKernelGGL(reduce_kernel<S>, g, dim3(256), 0, st, disp, W, H, ncols, m.D,
                       m.reduce_mode, m.sub, q);
}

hipError_t launch_reduce(const DeviceModel& m, const float* disp, int W, int H, int ncols,
                         int16_t* q, hipStream_t st) {
    const dim3 g((ncols + 63) / 64, (H + 15) / 16);
    switch (m.s) {
#define STX_CASE(n) case n: reduce_launch<n>(g, m, disp, W, H, ncols, q, st); break;
        STX_CASE(1) STX_CASE(2) STX_CASE(3) STX_CASE(4) STX_CASE(5) STX_CASE(6) STX_CASE(7)
        STX_CASE(8) STX_CASE(9) STX_CASE(10) STX_CASE(11) STX_CASE(12) STX_CASE(13)
        STX_CASE(14) STX_CASE(15) STX_CASE(16)
#undef STX_CASE
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_tables(const DeviceModel& m, const FrameWorkspace& ws, int H, int ncols,
                         int vtop, hipStream_t st) {
    (void)vtop;
    TablesArgs a;
    a.q = ws.q;
    a.prefix = ws.prefix;
    a.range = ws.range;
    a.po = ws.po;
    a.sky = m.sky;
    a.ground = m.ground;
    a.object_t = m.object_t;
    a.obj_k = m.obj_k;
    a.c_out = m.c_out;
    a.online = m.object_online;
    a.g = m.g;
    a.sub = m.sub;
    a.H = H;
    a.ncols = ncols;
    a.D = m.D;
    hipLaunchKernelGGL(tables_kernel, dim3(ncols), dim3(512), 0, st, a);
    return hipGetLastError();
}

int frame_waves(int requested, int H, int ncols, int num_cu) {
    const int slots = kernel_slots(H);
    if (requested > 0) return std::min(requested, slots >= 4 ? 4 : (slots >= 2 ? 2 : 1));
    // automatic: one wave per column (a recurrence step is bound by the
    // latency of its gathers, which more waves do not shorten) unless the
    // frame has fewer columns than the device has compute units
    for (int w : {4, 2}) {
        if (w <= slots && (long long)ncols * w <= (long long)num_cu) return w;
    }
    return 1;
}

namespace {

// Largest POL dynamic LDS (bytes) of a variant on the current device, set
// once per variant as the kernel's limit; 0 if the device refuses.
int pol_lds_bytes(const void* f, int lds_per_block) {
    static std::mutex mu;
    static std::map<const void*, int> cache;
    std::lock_guard<std::mutex> lock(mu);
    auto it = cache.find(f);
    if (it != cache.end()) return it->second;
    hipFuncAttributes fa{};
    int b = 0;
    if (hipFuncGetAttributes(&fa, f) == hipSuccess) {
        b = lds_per_block - (int)fa.sharedSizeBytes;
        b = (b / 16) * 16;
        if (b <= 0 ||
            hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, b) != hipSuccess)
            b = 0;
    }
    cache[f] = b;
    return b;
}

}  // namespace

bool frame_po_lds(int placement, int H) {
    // automatic: LDS for columns of up to 512 rows (a table of up to about
    // 80 disparity rows then fits)
    return placement == 2 || (placement == 0 && kernel_slots(H) <= 8);
}

hipError_t launch_dp(const DeviceModel& m, const FrameWorkspace& ws, int H, int ncols, int vtop,
                     int waves, bool po_lds, int lds_per_block, const FrameOutput& out,
                     hipStream_t st) {
    DpArgs a;
    a.q = ws.q;
    a.object_df = m.object_df;
    a.prefix = ws.prefix;
    a.range = ws.range;
    a.po = ws.po;
    a.fg_hi = m.fg_hi;
    a.fg_lo = m.fg_lo;
    a.counts = out.counts;
    a.records = out.records;
    a.total = out.total;
    a.overflow = out.overflow;
    a.cap = out.cap;
    a.H = H;
    a.ncols = ncols;
    a.D = m.D;
    a.vtop = vtop;
    a.lds_floats = 0;
    a.prior = m.prior;
    const int slots = kernel_slots(H), nch = kernel_chunks(m.D);
    // the LDS copy exists for one wave per column and d_range <= 128 only:
    // with both recurrences in one kernel the other variants run out of
    // registers, and they were not faster with it
    if (po_lds) {
        if (const void* f = dp_kernel_ptr(slots, nch, waves, true)) {
            const int bytes = pol_lds_bytes(f, lds_per_block);
            if (bytes > 0) {
                a.lds_floats = bytes / 4;
                void* args[] = {&a};
                return hipLaunchKernel(f, dim3(ncols), dim3(64 * waves), args, (size_t)bytes, st);
            }
        }
    }
    const void* f = dp_kernel_ptr(slots, nch, waves, false);
    if (!f) return hipErrorInvalidValue;
    void* args[] = {&a};
    return hipLaunchKernel(f, dim3(ncols), dim3(64 * waves), args, 0, st);
}

hipError_t run_selftest_mean(int D, int max_height, int64_t* mismatches) {
    unsigned long long* d_bad = nullptr;
    hipError_t e = hipMalloc(&d_bad, sizeof(unsigned long long));
    if (e != hipSuccess) return e;
    e = hipMemset(d_bad, 0, sizeof(unsigned long long));
    if (e == hipSuccess) {
        const float eps = (float)ldexp((double)D, -22);
        hipLaunchKernelGGL(selftest_mean_kernel, dim3(max_height + 1), dim3(256), 0, nullptr, D, eps,
                           d_bad);
        e = hipGetLastError();
    }
    unsigned long long h = 0;
    if (e == hipSuccess) e = hipMemcpy(&h, d_bad, sizeof(h), hipMemcpyDeviceToHost);
    (void)hipFree(d_bad);
    *mismatches = (int64_t)h;
    return e;
}

}  // namespace stx
