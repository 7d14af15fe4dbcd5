// dp_kernel.h -- the recurrence kernel of the staged per-frame path (Sec.
// 4.3-4.4): one workgroup of W wave64s per column, reading the column's
// prefix tables written by the tables kernel.  Instantiated per slot count
// in the inst_s*.hip units (kernel_table.h).
#pragma once

#include "dp_column.h"

namespace stx {

// ------------------------------------------------------------------ dp
struct DpArgs {
    const int16_t* q;
    const float* object_df;
    const float* prefix;
    const int32_t* range;
    const float* po;
    const int32_t* fg_hi;
    const int32_t* fg_lo;
    int32_t* counts;
    uint32_t* records;
    float* total;
    uint8_t* overflow;
    int cap, H, ncols, D, vtop;
    int lds_floats;         // dynamic LDS of a POL launch, in floats
    Prior prior;
};

// n floats from global memory into LDS by the W waves of the workgroup, and
// a barrier.  The 16-byte-aligned body goes through direct global-to-LDS
// loads (lane l of a wave fills bytes [16 l, 16 l + 16) above the wave's
// LDS base; no register round trip, many loads in flight); the tail, and a
// source that is not 16-byte aligned, through ordinary loads.  Nothing past
// g[n-1] is read.
template <int W>
__device__ void copy_to_lds(float* lds, const float* g, int n) {
    const int lane = threadIdx.x & 63;
    const int wave = (W == 1) ? 0 : __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    int done = 0;
    if ((reinterpret_cast<uintptr_t>(g) & 15u) == 0) {
        const int n4 = n & ~3;
        for (int base = wave * 256; base < n4; base += 256 * W) {
            const int i = base + 4 * lane;
            if (i < n4)
                __builtin_amdgcn_global_load_lds(g + i,
                                                 (__attribute__((address_space(3))) void*)(lds + base),
                                                 16, 0, 0);
        }
        done = n4;
    }
    for (int i = done + (int)threadIdx.x; i < n; i += 64 * W) lds[i] = g[i];
    __builtin_amdgcn_s_waitcnt(0);   // the direct loads have landed
    __syncthreads();
}

// One workgroup of W waves per column.  POL: the column's object prefix
// table is copied into dynamic LDS when it fits (one copy, contiguous rows),
// so that the recurrence gathers from LDS instead of the caches and HBM.
template <int S, int NCH, int W, bool POL>
__global__ __launch_bounds__(64 * W) void dp_kernel(DpArgs a) {
    __shared__ ColumnLds<S, W, 64 * NCH> lds;
    // the column's reduced pixels live in the object row-cost array, which
    // solve_column writes only after its last read of them
    int16_t* const qs = reinterpret_cast<int16_t*>(lds.crow_o);
    const int col = blockIdx.x;
    const int stride = a.H + 1;
    for (int v = threadIdx.x; v < a.H; v += 64 * W) qs[v] = a.q[(size_t)col * a.H + v];
    __syncthreads();
    ColumnIn in;
    in.PG = a.prefix + ((size_t)0 * a.ncols + col) * stride;
    in.PS = a.prefix + ((size_t)1 * a.ncols + col) * stride;
    in.PA = a.prefix + ((size_t)2 * a.ncols + col) * stride;
    in.PN2 = a.prefix + ((size_t)3 * a.ncols + col) * stride;
    in.PO = a.po + (size_t)col * a.D * stride;
    in.fbase = a.range[2 * col];
    in.fmax = a.range[2 * col + 1];
    in.q = qs;
    in.O_df = a.object_df;
    in.D = a.D;
    in.fg_hi = a.fg_hi;
    in.fg_lo = a.fg_lo;
    ColumnOut out;
    out.count = a.counts + col;
    out.rec = a.records + (size_t)col * a.cap * 3;
    out.total = a.total + col;
    out.overflow = a.overflow + col;
    out.cap = a.cap;
    if constexpr (POL) {
        extern __shared__ float po_lds[];
        const int n = (in.fmax - in.fbase + 1) * stride;   // uniform over the workgroup
        if (n <= a.lds_floats) {
            copy_to_lds<W>(po_lds, in.PO, n);
            solve_column<S, NCH, W, true, false>(a.H, a.vtop, a.prior, in, out, lds, po_lds);
            return;
        }
    }
    solve_column<S, NCH, W, false, false>(a.H, a.vtop, a.prior, in, out, lds);
}

}  // namespace stx
