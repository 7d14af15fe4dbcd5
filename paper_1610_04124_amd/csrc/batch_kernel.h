// batch_kernel.h -- the persistent fused kernel of the batched launch.
//
// Every (frame, column) pair is a task.  The host orders tasks by decreasing
// frame height (the recurrence costs O(h^2) per column, Sec. 3.3), so the
// longest columns start first, and resident workgroups pull tasks from a
// device counter until the list is exhausted.  Each task runs the whole
// per-column pipeline of Sec. 4 without leaving the workgroup: strip
// reduction into LDS, the prefix tables and object prefix rows into the
// workgroup's own scratch slot (written and re-read by the same workgroup,
// so they stay in L2), then the recurrence and backtracking of dp_column.h.
// Results are bit-identical to the per-frame kernels: the arithmetic is the
// same exact grid arithmetic, only the schedule differs.
//
// The templates are instantiated per slot count in the inst_s*.hip units
// (kernel_table.h), so that the variants compile in parallel.
#pragma once

#include <climits>

#include "dp_column.h"

namespace stx {

// A named namespace (not an anonymous one) so that profilers show the
// kernels by name.
namespace persist {

struct JobDesc {
    const float* disp;
    const float* sky;
    const float* ground;
    const float* object_t;
    const float* object_df;
    const int32_t* fg_hi;
    const int32_t* fg_lo;
    int32_t* counts;
    uint32_t* records;
    float* total;
    uint8_t* overflow;
    int W, H, s, ncols, D, vtop, reduce_mode, cap;
    int sub;              // disparity bins of 2^-sub px
    Prior prior;
    // shader-clock cycles per task phase, summed over the launch (builds
    // with STX_PHASE_TIMING only; null and unused otherwise)
    unsigned long long* phase;
};

// Phases of a column task timed by STX_PHASE_TIMING builds: reduction (with
// the column's disparity range), the four small prefix scans, the object
// prefix table, the recurrence, the backtracking; then the task count and
// the workgroups' summed lifetime (start delay and final waits included).
enum PhaseSlot {
    kPhaseReduce = 0, kPhaseScans, kPhaseObjectTable, kPhaseRecurrence, kPhaseBacktrack,
    kPhaseTasks, kPhaseLifetime, kPhaseSlots = 8
};

// Scratch slot of one column task (floats): the ground, sky, disparity-sum
// and count prefixes (H+1 each), then the object prefix rows.  Entry i of an
// object row sits at float i + 3 of a 16-byte aligned row of
// slot_row_floats(H) floats, so that entries 4l+1 .. 4l+4 (the prefixes a
// lane holding rows 4l .. 4l+3 produces) form one aligned 16-byte store; the
// row leaves room for a lane whose rows run past H.
__host__ __device__ constexpr long long slot_row_floats(int H) { return ((H + 10) / 4) * 4; }
__host__ __device__ constexpr long long slot_rows_offset(int H) { return ((4LL * (H + 1) + 3) / 4) * 4; }
__host__ __device__ constexpr long long slot_floats(int H, int D) {
    // the full table (D rows of slot_row_floats) or the banded one (per
    // 64-row slot at most D rows and the +inf row, 64 floats each)
    return slot_rows_offset(H) + ((long long)D * slot_row_floats(H) > 64LL * ((H + 63) / 64) * (D + 1)
                                      ? (long long)D * slot_row_floats(H)
                                      : 64LL * ((H + 63) / 64) * (D + 1));
}

// The persistent kernel keeps a banded object prefix table (solve_column's
// BAND) for costs on the grid; the recurrence with links for costs off the
// grid keeps the full table.
template <int S, int W, bool LINKS>
constexpr bool kBanded = !LINKS;

__device__ __forceinline__ int reduce_any(const float* p, int s, int mode, int D, int sub) {
    switch (s) {
#define STX_CASE(n) case n: return reduce_strip<n>(p, mode, D, sub);
        STX_CASE(1) STX_CASE(2) STX_CASE(3) STX_CASE(4) STX_CASE(5) STX_CASE(6) STX_CASE(7)
        STX_CASE(8) STX_CASE(9) STX_CASE(10) STX_CASE(11) STX_CASE(12) STX_CASE(13)
        STX_CASE(14) STX_CASE(15) STX_CASE(16)
#undef STX_CASE
        default: return -1;
    }
}

__device__ __forceinline__ int wave_min_i(int x) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x = min(x, __shfl_xor(x, o, 64));
    return x;
}
__device__ __forceinline__ int wave_max_i(int x) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x = max(x, __shfl_xor(x, o, 64));
    return x;
}

// Start delay between consecutive XCDs of a long batched launch, in shader
// clock cycles (~5 us).
constexpr unsigned int kXcdStaggerCycles = 10000u;

// Waves per SIMD the register allocation of each variant is held to (the
// compiler's own choice leaves a few registers above the next step down).
// Columns of up to 7 slots per wave get 128 registers (4 waves per SIMD):
// with the banded object prefix table, one-wave columns held to 96 (5 waves)
// spilled more and measured 4 % slower.
constexpr int batch_waves(int slots_per_wave, int waves) {
    (void)waves;
    return slots_per_wave <= 7 ? 4 : (slots_per_wave <= 14 ? 3 : 2);
}

// One workgroup of W waves per column task.  LINKS: the recurrence keeps
// its links and the backtracking follows them (costs off the grid).
template <int S, int NCH, int W, bool LINKS = false>
__global__ __launch_bounds__(64 * W)
__attribute__((amdgpu_waves_per_eu(batch_waves((S + W - 1) / W, W)))) void batch_kernel(
    const JobDesc* __restrict__ jobs, const int2* __restrict__ tasks, int ntasks,
    unsigned int* counter, float* scratch, long long scratch_stride, int hmax,
    unsigned int stagger) {
    __shared__ ColumnLds<S, W, 64 * NCH, LINKS> lds;
    // the column's reduced pixels live in the object row-cost array, which
    // solve_column writes only after its last read of them
    int16_t* const qs = reinterpret_cast<int16_t*>(lds.crow_o);
    // per wave: one row of the object cost table while its prefix row is
    // built, and a zero (the cost of an invalid pixel) after it
    __shared__ float ostage[W][64 * NCH + 4];
    constexpr bool BAND = kBanded<S, W, LINKS>;
    // BAND, per slot: first and last mean of its band, float offset of its rows
    __shared__ int band_lo[S], band_hi[S], band_base[S], band_all[3];
    __shared__ int task_slot;
    __shared__ int red[3][W];
    // one-wave banded columns of up to 8 slots: rcp(2 n) for n = 0 .. 64 S,
    // read by the recurrence in place of a v_rcp_f32 per candidate (the same
    // values; rcp(0) = +inf); written once per workgroup, before the first
    // task's barriers
    constexpr bool RT = BAND && W == 1 && S <= 8;
    __shared__ float rtab[RT ? 64 * S + 1 : 1];
    const int lane = threadIdx.x & 63;
    const int wave = (W == 1) ? 0 : __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    float* ws = scratch + (size_t)blockIdx.x * (size_t)scratch_stride;
    (void)hmax;
    if constexpr (RT) {
        for (int n = threadIdx.x; n <= 64 * S; n += 64 * W)
            rtab[n] = __builtin_amdgcn_rcpf((float)(2 * n));
    }
#ifdef STX_PHASE_TIMING
    // wave 0 stamps the shader clock at each phase boundary of a task
    const unsigned long long t_entry = __builtin_amdgcn_s_memtime();
    unsigned long long* phase_acc = nullptr;
    __shared__ unsigned long long t_rec_end;
    auto phase_add = [&](int slot, unsigned long long v) {
        if (threadIdx.x == 0 && phase_acc) atomicAdd(phase_acc + slot, v);
    };
#endif
    // Workgroups are dispatched to the eight XCDs in turn.  When every
    // column takes equally long, all of them would reach the memory-heavy
    // table builds together, round after round; starting XCD x stagger * x
    // cycles late spreads those bursts over the shared memory system
    // (measured: 2 % at 1024x440 with five waves per SIMD; with the banded
    // tables and four waves per SIMD, 0 to 20,000 cycles all within 1 %).
    if (stagger != 0u) {
        const unsigned int xcd = blockIdx.x & 7u;
        const unsigned long long t0 = __builtin_amdgcn_s_memtime();
        const unsigned long long dl = (unsigned long long)xcd * stagger;
        while (__builtin_amdgcn_s_memtime() - t0 < dl) __builtin_amdgcn_s_sleep(127);
    }
    for (;;) {
        int t = 0;
        if constexpr (W == 1) {
            if (lane == 0) t = (int)atomicAdd(counter, 1u);
            t = __builtin_amdgcn_readfirstlane(t);
        } else {
            if (threadIdx.x == 0) task_slot = (int)atomicAdd(counter, 1u);
            __syncthreads();
            t = __builtin_amdgcn_readfirstlane(task_slot);
        }
        if (t >= ntasks) break;
        const int2 tk = tasks[t];
        const JobDesc& J = jobs[tk.x];
        const int H = J.H, D = J.D, col = tk.y, stride = H + 1;
#ifdef STX_PHASE_TIMING
        phase_acc = J.phase;
        const unsigned long long t0 = __builtin_amdgcn_s_memtime();
#endif

        // Sec. 4.1: reduce this column's strips, bottom-up, into LDS
        int lmin = INT_MAX, lmax = -1;
        bool inv = false;
        for (int v = threadIdx.x; v < H; v += 64 * W) {
            const int r = H - 1 - v;
            const int x = reduce_any(J.disp + (size_t)r * J.W + (size_t)col * J.s, J.s,
                                     J.reduce_mode, D, J.sub);
            qs[v] = (int16_t)x;
            if (x >= 0) {
                lmin = min(lmin, x);
                lmax = max(lmax, x);
            } else {
                inv = true;
            }
        }
        // object means lie in [smallest, largest valid q]; a stixel without
        // valid pixels has mean 0, so the table starts at 0 when the column
        // holds an invalid pixel
        int anyinv = __ballot(inv) ? 1 : 0;
        int fmin = wave_min_i(lmin);
        int fmax = wave_max_i(lmax);
        if constexpr (W > 1) {
            if (lane == 0) {
                red[0][wave] = fmin;
                red[1][wave] = fmax;
                red[2][wave] = anyinv;
            }
            __syncthreads();
#pragma unroll
            for (int w = 0; w < W; ++w) {
                fmin = min(fmin, red[0][w]);
                fmax = max(fmax, red[1][w]);
                anyinv |= red[2][w];
            }
        }
        if (anyinv) fmin = 0;
        if (fmax < 0) {
            fmin = 0;
            fmax = 0;
        }
        // the same in every lane; reading them from the first lane lets the
        // compiler keep them (and the row offsets derived from them) scalar
        fmin = __builtin_amdgcn_readfirstlane(fmin);
        fmax = __builtin_amdgcn_readfirstlane(fmax);
        __syncthreads();
#ifdef STX_PHASE_TIMING
        const unsigned long long t1 = __builtin_amdgcn_s_memtime();
        unsigned long long t2 = t1;
#endif

        // Sec. 4.2: prefix tables into the scratch slot: the four small ones
        // by wave 0, the object rows f = fmin + wave, fmin + wave + W, ...
        // Every load of a table row (one per 64-row slot) is issued before
        // its scan starts, so a row costs one memory latency rather than one
        // per slot.
        float* PG = ws;
        float* PS = ws + stride;
        float* PA = ws + 2 * stride;
        float* PN = ws + 3 * stride;
        float* PO = ws + slot_rows_offset(H);
        const int pstride = (int)slot_row_floats(H);
        const int nsl = (H + 63) >> 6;
        auto q_at = [&](int c) {
            const int v = 64 * c + lane;
            return (v < H) ? (int)qs[v] : -1;
        };
        if (wave == 0) {
            if (lane == 0) {
                PG[0] = 0.0f;
                PS[0] = 0.0f;
                PA[0] = 0.0f;
                PN[0] = 0.0f;
            }
            float cg = 0.0f, cs = 0.0f, ca = 0.0f, cn = 0.0f;
            for (int c = 0; c < nsl; ++c) {
                const int v = 64 * c + lane, x = q_at(c);
                float g = 0.0f, sk = 0.0f, aa = 0.0f, nn = 0.0f;
                if (x >= 0) {
                    g = J.ground[(size_t)(H - 1 - v) * D + x];
                    sk = J.sky[x];
                    aa = (float)(2 * x + 1);
                    nn = 2.0f;
                }
                g = wave_inclusive_scan(g) + cg;
                sk = wave_inclusive_scan(sk) + cs;
                aa = wave_inclusive_scan(aa) + ca;
                nn = wave_inclusive_scan(nn) + cn;
                if (v < H) {
                    PG[v + 1] = g;
                    PS[v + 1] = sk;
                    PA[v + 1] = aa;
                    PN[v + 1] = nn;
                }
                cg = readlane_f(g, 63);
                cs = readlane_f(sk, 63);
                ca = readlane_f(aa, 63);
                cn = readlane_f(nn, 63);
            }
#ifdef STX_PHASE_TIMING
            __builtin_amdgcn_s_waitcnt(0);
            t2 = __builtin_amdgcn_s_memtime();
#endif
        }
        uint32_t po_bytes = 0;
        if constexpr (BAND) {
            // Bands: a stixel [b, k] with k in slot t and a valid pixel has a
            // mean between the smallest and the largest of (a) the valid
            // pixels of slot t and (b) the means of the stixels [b', 64t-1]
            // (b' < 64 t) with a valid pixel: its mean is a weighted average
            // of the mean of its part below the slot and that of its part in
            // the slot, and rounding is monotone.
            __syncthreads();   // wave 0's prefix tables are read back below
            int glo = INT_MAX, ghi = -1, base = 0;
            if (wave == 0) {
#pragma unroll
            for (int t = 0; t < S; ++t) {
                if (64 * t >= H) {
                    // padding: the recurrence's reads of this slot stay in range
                    if (lane == 0) {
                        band_lo[t] = fmin;
                        band_hi[t] = -1;
                        band_base[t] = 0;
                    }
                    continue;
                }
                const int x = q_at(t);
                int lo = (x >= 0) ? x : INT_MAX, hi = x;
                if (t > 0) {
                    const float ax = PA[64 * t], nx = PN[64 * t];
                    for (int c = 0; c < t; ++c) {
                        const int b0 = 64 * c + lane;
                        const float n2 = nx - PN[b0];
                        if (n2 != 0.0f) {
                            const int f = mean_index(ax - PA[b0], n2, J.prior.mean_eps);
                            lo = min(lo, f);
                            hi = max(hi, f);
                        }
                    }
                }
                lo = wave_min_i(lo);
                hi = wave_max_i(hi);
                if (hi < 0) lo = hi = fmin;     // no valid pixel reaches the slot
                lo = __builtin_amdgcn_readfirstlane(lo);
                hi = __builtin_amdgcn_readfirstlane(hi);
                if (lane == 0) {
                    band_lo[t] = lo;
                    band_hi[t] = hi;
                    band_base[t] = base;
                }
                // the +inf row (stixels without a valid pixel read it)
                buf_store_b(make_rsrc(PO, 0x7ffffff0u), inf_f(), (uint32_t)(base + lane) * 4u, 0u);
                base += (hi - lo + 2) * 64;
                glo = min(glo, lo);
                ghi = max(ghi, hi);
            }
            if (W > 1 && lane == 0) {
                band_all[0] = glo;
                band_all[1] = ghi;
                band_all[2] = base;
            }
            }
            __syncthreads();
            if constexpr (W > 1) {
                glo = __builtin_amdgcn_readfirstlane(band_all[0]);
                ghi = __builtin_amdgcn_readfirstlane(band_all[1]);
                base = __builtin_amdgcn_readfirstlane(band_all[2]);
            }
            po_bytes = (uint32_t)base * 4u;
            // Object rows f in [glo, ghi]: the full prefix over the column is
            // scanned as in the full table, but a lane stores its four
            // prefixes only where f lies in its slot's band, at row
            // f - lo + 1 of the band.
            constexpr int U = (64 * S + 255) / 256;
            constexpr int NST = 64 * NCH;
            float* const stg = ostage[wave];
            if (lane == 0) stg[NST] = 0.0f;
            int qi[U][4];
            int slo[U], shi[U], sbase[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int v = 256 * u + 4 * lane + i;
                    const int x = (v < H) ? (int)qs[v] : -1;
                    qi[u][i] = (x >= 0) ? x : NST;
                }
                const int t = min(4 * u + (lane >> 4), S - 1);
                const bool real = (256 * u + 4 * lane) < 64 * S;
                slo[u] = band_lo[t];
                shi[u] = real ? band_hi[t] : -1;
                // float offset of entry (mean f, position 4 (lane mod 16)) is
                // sbase + 64 f: the band's rows start one row below mean lo
                sbase[u] = band_base[t] + 64 * (1 - band_lo[t]) + 4 * (lane & 15);
            }
            const auto otr = make_rsrc(J.object_t, (uint32_t)(D * D) * 4u);
            const auto pow_ = make_rsrc(PO, po_bytes);
            float onext[NCH];
            auto load_costs = [&](int f) {
                const uint32_t rowb = (uint32_t)(f * D) * 4u;
#pragma unroll
                for (int c = 0; c < NCH; ++c) onext[c] = buf_load_b(otr, (uint32_t)(64 * c + lane) * 4u, rowb);
            };
            if (W == 1 || glo + wave <= ghi) load_costs(glo + wave);   // glo <= ghi
#pragma unroll 1
            for (int f = glo + wave; f <= ghi; f += W) {
#pragma unroll
                for (int c = 0; c < NCH; ++c) stg[64 * c + lane] = onext[c];
                if (f + W <= ghi) load_costs(f + W);
                float carry = 0.0f;
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    if (256 * u >= H) break;
                    const float o0 = stg[qi[u][0]], o1 = stg[qi[u][1]];
                    const float o2 = stg[qi[u][2]], o3 = stg[qi[u][3]];
                    const float a1 = o0 + o1, a2 = a1 + o2, a3 = a2 + o3;
                    const float incl = wave_inclusive_scan(a3);
                    const float e = (incl - a3) + carry;
                    const float r0 = e + o0, r1 = e + a1, r2 = e + a2, r3 = e + a3;
                    if (f >= slo[u] && f <= shi[u])
                        buf_store_b4(pow_, r0, r1, r2, r3, (uint32_t)(sbase[u] + 64 * f) * 4u, 0u);
                    carry = readlane_f(incl, 63) + carry;
                }
            }
        } else {
        // The object rows f = fmin + wave, fmin + wave + W, ...: row f of the
        // object cost table (costs of mean f for every pixel disparity) is
        // staged in LDS with a few coalesced loads; lane l then takes the
        // costs of rows 256u + 4l .. 256u + 4l + 3 from it (a zero for an
        // invalid pixel or a row past H), sums them in order, adds the wave
        // scan of the lanes' sums and stores its four prefixes with one
        // aligned 16-byte store.  The next row's loads are in flight while a
        // row is scanned.
        constexpr int U = (64 * S + 255) / 256;     // 256-row groups
        constexpr int NST = 64 * NCH;               // staged costs per row
        float* const stg = ostage[wave];
        if (lane == 0) stg[NST] = 0.0f;
        int qi[U][4];                               // index of each row's cost in the stage
#pragma unroll
        for (int u = 0; u < U; ++u) {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int v = 256 * u + 4 * lane + i;
                const int x = (v < H) ? (int)qs[v] : -1;
                qi[u][i] = (x >= 0) ? x : NST;
            }
        }
        const auto otr = make_rsrc(J.object_t, (uint32_t)(D * D) * 4u);
        const auto pow_ = make_rsrc(PO, (uint32_t)(fmax - fmin + 1) * (uint32_t)pstride * 4u);
        float onext[NCH];
        auto load_costs = [&](int f) {
            const uint32_t rowb = (uint32_t)(f * D) * 4u;
#pragma unroll
            for (int c = 0; c < NCH; ++c) onext[c] = buf_load_b(otr, (uint32_t)(64 * c + lane) * 4u, rowb);
        };
        if (fmin + wave <= fmax) load_costs(fmin + wave);
#pragma unroll 1
        for (int f = fmin + wave; f <= fmax; f += W) {
#pragma unroll
            for (int c = 0; c < NCH; ++c) stg[64 * c + lane] = onext[c];
            if (f + W <= fmax) load_costs(f + W);
            const uint32_t rowoff = (uint32_t)(f - fmin) * (uint32_t)pstride * 4u;
            if (lane == 0) buf_store_b(pow_, 0.0f, 12u, rowoff);
            float carry = 0.0f;
#pragma unroll
            for (int u = 0; u < U; ++u) {
                if (256 * u >= H) break;
                const float o0 = stg[qi[u][0]], o1 = stg[qi[u][1]];
                const float o2 = stg[qi[u][2]], o3 = stg[qi[u][3]];
                const float a1 = o0 + o1, a2 = a1 + o2, a3 = a2 + o3;
                const float incl = wave_inclusive_scan(a3);
                const float e = (incl - a3) + carry;
                const float r0 = e + o0, r1 = e + a1, r2 = e + a2, r3 = e + a3;
                if (256 * u + 4 * lane < H)
                    buf_store_b4(pow_, r0, r1, r2, r3, (uint32_t)(1024 * u + 16 * lane + 16), rowoff);
                carry = readlane_f(incl, 63) + carry;
            }
        }
        }
        __syncthreads();   // the tables written above are read back below, by every wave
#ifdef STX_PHASE_TIMING
        const unsigned long long t3 = __builtin_amdgcn_s_memtime();
#endif

        // Sec. 4.3-4.4
        ColumnIn in;
        in.PG = PG;
        in.PS = PS;
        in.PA = PA;
        in.PN2 = PN;
        if constexpr (BAND) {
            in.PO = PO;
            in.band_lo = band_lo;
            in.band_base = band_base;
            in.po_bytes = po_bytes;
            in.rtab = rtab;
        } else {
            in.PO = PO + 3;
            in.po_stride = pstride;
        }
        in.fbase = fmin;
        in.fmax = fmax;
        in.q = qs;
        in.O_df = J.object_df;
        in.D = D;
        in.fg_hi = J.fg_hi;
        in.fg_lo = J.fg_lo;
        in.S_tab = J.sky;
        in.G_tab = J.ground;
        ColumnOut out;
        out.count = J.counts + col;
        out.rec = J.records + (size_t)col * J.cap * 3;
        out.total = J.total + col;
        out.overflow = J.overflow + col;
        out.cap = J.cap;
#ifdef STX_PHASE_TIMING
        out.t_rec_end = &t_rec_end;
#endif
        solve_column<S, NCH, W, false, true, LINKS, BAND, RT>(H, J.vtop, J.prior, in, out, lds);
#ifdef STX_PHASE_TIMING
        if (threadIdx.x == 0) {
            __builtin_amdgcn_s_waitcnt(0);
            const unsigned long long t5 = __builtin_amdgcn_s_memtime();
            phase_add(kPhaseReduce, t1 - t0);
            phase_add(kPhaseScans, t2 - t1);
            phase_add(kPhaseObjectTable, t3 - t2);
            phase_add(kPhaseRecurrence, t_rec_end - t3);
            phase_add(kPhaseBacktrack, t5 - t_rec_end);
            phase_add(kPhaseTasks, 1ull);
        }
#endif
        __syncthreads();   // every read of the slot completes before the next task rewrites it
    }
#ifdef STX_PHASE_TIMING
    phase_add(kPhaseLifetime, __builtin_amdgcn_s_memtime() - t_entry);
#endif
}

// Sec. 4.1-4.2 for one column by one wave: its strips reduced into qs (LDS,
// bottom-up; -1 past H and for a column that does not exist), then its
// prefix tables at ws (PG, PS, PA, PN at 0..3 (h+1), the object rows from
// po_at floats on).  Returns the column's disparity range [fmin, fmax].
template <int S>
__device__ __forceinline__ void column_tables(const JobDesc& J, const int col, const bool exists, int16_t* qs,
                              float* ws, const int po_at, int& fmin_out, int& fmax_out) {
    const int lane = threadIdx.x & 63;
    const int H = J.H, D = J.D, stride = H + 1;
    int lmin = INT_MAX, lmax = -1;
    bool inv = false;
    for (int v = lane; v < 64 * S; v += 64) {
        int x = -1;
        if (exists && v < H)
            x = reduce_any(J.disp + (size_t)(H - 1 - v) * J.W + (size_t)col * J.s, J.s,
                           J.reduce_mode, D, J.sub);
        qs[v] = (int16_t)x;
        if (x >= 0) {
            lmin = min(lmin, x);
            lmax = max(lmax, x);
        } else if (v < H) {
            inv = true;
        }
    }
    int fmin = __ballot(inv) ? 0 : wave_min_i(lmin);
    int fmax = wave_max_i(lmax);
    if (fmax < 0) {
        fmin = 0;
        fmax = 0;
    }
    fmin = __builtin_amdgcn_readfirstlane(fmin);
    fmax = __builtin_amdgcn_readfirstlane(fmax);
    fmin_out = fmin;
    fmax_out = fmax;
    __syncthreads();
    float* PG = ws;
    float* PS = ws + stride;
    float* PA = ws + 2 * stride;
    float* PN = ws + 3 * stride;
    if (lane == 0) {
        PG[0] = 0.0f;
        PS[0] = 0.0f;
        PA[0] = 0.0f;
        PN[0] = 0.0f;
    }
    float cg = 0.0f, cs = 0.0f, ca = 0.0f, cn = 0.0f;
    for (int base = 0; base < H; base += 64) {
        const int v = base + lane;
        const int x = (v < H) ? (int)qs[v] : -1;
        float g = 0.0f, sk = 0.0f, aa = 0.0f, nn = 0.0f;
        if (x >= 0) {
            g = J.ground[(size_t)(H - 1 - v) * D + x];
            sk = J.sky[x];
            aa = (float)(2 * x + 1);
            nn = 2.0f;
        }
        g = wave_inclusive_scan(g) + cg;
        sk = wave_inclusive_scan(sk) + cs;
        aa = wave_inclusive_scan(aa) + ca;
        nn = wave_inclusive_scan(nn) + cn;
        if (v < H) {
            PG[v + 1] = g;
            PS[v + 1] = sk;
            PA[v + 1] = aa;
            PN[v + 1] = nn;
        }
        cg = readlane_f(g, 63);
        cs = readlane_f(sk, 63);
        ca = readlane_f(aa, 63);
        cn = readlane_f(nn, 63);
    }
    const auto otr = make_rsrc(J.object_t, (uint32_t)(D * D) * 4u);
    const auto pow_ =
        make_rsrc(ws + po_at, (uint32_t)(fmax - fmin + 1) * (uint32_t)stride * 4u);
    uint32_t qoff[S];
#pragma unroll
    for (int c = 0; c < S; ++c) {
        const int v = 64 * c + lane;
        const int x = (v < H) ? (int)qs[v] : -1;
        qoff[c] = (x >= 0) ? (uint32_t)x * 4u : 0x40000000u;
    }
#pragma unroll 1
    for (int f = fmin; f <= fmax; ++f) {
        const uint32_t rowb = (uint32_t)(f * D) * 4u;
        float oc[S];
#pragma unroll
        for (int c = 0; c < S; ++c) oc[c] = buf_load_b(otr, qoff[c], rowb);
        const uint32_t rowoff = (uint32_t)(f - fmin) * (uint32_t)stride * 4u;
        if (lane == 0) buf_store_b(pow_, 0.0f, 0u, rowoff);
        float carry = 0.0f;
#pragma unroll
        for (int c = 0; c < S; ++c) {
            const int v = 64 * c + lane;
            const float o = wave_inclusive_scan(oc[c]) + carry;
            if (v < H) buf_store_b(pow_, o, (uint32_t)(v + 1) * 4u, rowoff);
            carry = readlane_f(o, 63);
        }
    }
}

// Two columns of one frame per one-wave workgroup (solve_pair): tasks are
// (frame, even column) pairs.  The workgroup's scratch slot holds the two
// columns' tables one column stride ((8 + D)(h+1) floats) apart.
template <int S, int NCH>
__global__ __launch_bounds__(64)
__attribute__((amdgpu_waves_per_eu(3))) void batch_pair_kernel(
    const JobDesc* __restrict__ jobs, const int2* __restrict__ tasks, int ntasks,
    unsigned int* counter, float* scratch, long long scratch_stride, int hmax) {
    __shared__ int16_t qs2[2 * 64 * S];
    __shared__ float qtab2[2 * 256];
    __shared__ ColumnLds<S, 1> lds;
    const int lane = threadIdx.x;
    float* ws = scratch + (size_t)blockIdx.x * (size_t)scratch_stride;
    (void)hmax;
    for (;;) {
        int t = 0;
        if (lane == 0) t = (int)atomicAdd(counter, 1u);
        t = __builtin_amdgcn_readfirstlane(t);
        if (t >= ntasks) break;
        const int2 tk = tasks[t];
        const JobDesc& J = jobs[tk.x];
        const int H = J.H, D = J.D, col0 = tk.y, stride = H + 1;
        const bool has1 = col0 + 1 < J.ncols;
        const long long colstride = (long long)(8 + D) * stride;
        int fmin0, fmax0, fmin1, fmax1;
        column_tables<S>(J, col0, true, qs2, ws, 8 * stride, fmin0, fmax0);
        column_tables<S>(J, col0 + 1, has1, qs2 + 64 * S, ws + colstride, 8 * stride, fmin1,
                         fmax1);
        __syncthreads();   // the tables written above are read back below

        ColumnIn in0, in1;
        for (int x = 0; x < 2; ++x) {
            ColumnIn& in = x ? in1 : in0;
            float* base = ws + x * colstride;
            in.PG = base;
            in.PS = base + stride;
            in.PA = base + 2 * stride;
            in.PN2 = base + 3 * stride;
            in.rowc = base + 4 * stride;
            in.PO = base + 8 * stride;
            in.fbase = x ? fmin1 : fmin0;
            in.fmax = x ? fmax1 : fmax0;
            in.q = qs2 + x * 64 * S;
            in.O_df = J.object_df;
            in.D = D;
            in.fg_hi = J.fg_hi;
            in.fg_lo = J.fg_lo;
        }
        ColumnOut out0, out1;
        for (int x = 0; x < 2; ++x) {
            ColumnOut& out = x ? out1 : out0;
            const int col = col0 + x;
            out.count = J.counts + col;
            out.rec = J.records + (size_t)col * J.cap * 3;
            out.total = J.total + col;
            out.overflow = J.overflow + col;
            out.cap = J.cap;
        }
        solve_pair<S, NCH>(H, J.vtop, J.prior, in0, in1, out0, out1, has1, qs2, qtab2, lds);
        __syncthreads();   // every read of the slot completes before the next task rewrites it
    }
}

}  // namespace persist
}  // namespace stx
