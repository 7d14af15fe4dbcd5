// sgm.hip -- semi-global matching on gfx950: the stereo stage whose
// disparity maps feed the stixel path.  The paper takes its disparity from a
// GPU semi-global matching with census costs (Sec. 1, Sec. 5) and excludes
// that stage from its own timings; here it runs on the device ahead of the
// stixel kernels, so a stereo pair goes in and stixels come out with no host
// round trip.
//
// Method (Hirschmuller's semi-global matching, census costs):
//   census   9 x 7 window, bit i = 1 iff neighbour i (row-major, centre
//            skipped) lies inside the image and is darker than the centre
//   cost     C(p, d) = Hamming distance of left census (y, x) and right
//            census (y, x - d); 62 when x - d < 0
//   paths    L_r(p, d) = C(p, d) + min(L_r(p-r, d), L_r(p-r, d -+ 1) + P1,
//            M + P2) - M, M = min_k L_r(p-r, k); L_r = C at a path's start
//   select   d_L = smallest d of minimum summed cost; d_R(y, x) = smallest d
//            minimising S((y, x + d), d); left-right check |d_L - d_R| <= 1,
//            else -1 (the stixel input's invalid value)
//
// Work distribution: one wave64 per path line (an image row for the two
// horizontal directions, a column for the two vertical ones), lanes over
// disparities (lane l owns DPL consecutive disparities l DPL + i), steps
// along the line.  A step's neighbour terms d -+ 1 cross lanes by one DPP
// wavefront shift each; M is a DPP row minimum and three scalar minima.  The
// summed costs S live in HBM as uint16 [frame][y][x][d]: the top-to-bottom
// pass writes them, the bottom-to-top and right-to-left passes add to them,
// and the left-to-right pass, run last, adds its own term in registers and
// selects d_L (wave minimum of cost * 256 + d), keeps the right view's
// minima per target column in LDS (lane d of step x updates column x - d)
// and applies the left-right check once its row is done; S is never written
// back by that pass.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <new>
#include <string>
#include <type_traits>

#include "handle.h"
#include "internal.h"
#include "sgm.h"
#include "stixels.h"

namespace stx::sgm {

namespace {

constexpr int kCostOut = 62;
constexpr int kBig = 0x3fff;        // L of lanes past the disparity range
constexpr int kTileW = 64, kTileH = 16;

// ------------------------------------------------------------------ census
// blockIdx.z = 2 frame + side (0 left, 1 right).  The tile and its halo go
// through LDS; pixels outside the image are stored as 256, which is never
// darker than a centre.
__global__ __launch_bounds__(256) void census_kernel(const uint8_t* __restrict__ left,
                                                     const uint8_t* __restrict__ right, int W,
                                                     int H, uint64_t* __restrict__ cl,
                                                     uint64_t* __restrict__ cr) {
    __shared__ uint16_t tile[kTileH + 6][kTileW + 8];
    const int f = blockIdx.z >> 1, side = blockIdx.z & 1;
    const size_t off = (size_t)f * (size_t)W * (size_t)H;
    const uint8_t* img = (side ? right : left) + off;
    uint64_t* out = (side ? cr : cl) + off;
    const int x0 = blockIdx.x * kTileW, y0 = blockIdx.y * kTileH;
    for (int i = threadIdx.x; i < (kTileH + 6) * (kTileW + 8); i += 256) {
        const int ty = i / (kTileW + 8), tx = i - ty * (kTileW + 8);
        const int y = y0 + ty - 3, x = x0 + tx - 4;
        tile[ty][tx] = (y >= 0 && y < H && x >= 0 && x < W) ? img[(size_t)y * W + x] : 256;
    }
    __syncthreads();
    // thread (tx, g) takes the kTileH / 4 consecutive rows of group g in
    // column tx, keeping the 7 x 9 window in registers and reading one new
    // tile row per pixel (9 LDS reads instead of 63)
    constexpr int kRows = kTileH / 4;
    const int tx = threadIdx.x & 63;
    const int x = x0 + tx;
    const int r0 = (threadIdx.x >> 6) * kRows;
    int win[7][9];
#pragma unroll
    for (int dy = 0; dy < 6; ++dy) {
#pragma unroll
        for (int dx = 0; dx < 9; ++dx) win[dy + 1][dx] = tile[r0 + dy][tx + dx];
    }
#pragma unroll
    for (int k = 0; k < kRows; ++k) {
        const int r = r0 + k;
#pragma unroll
        for (int dy = 0; dy < 6; ++dy) {
#pragma unroll
            for (int dx = 0; dx < 9; ++dx) win[dy][dx] = win[dy + 1][dx];
        }
#pragma unroll
        for (int dx = 0; dx < 9; ++dx) win[6][dx] = tile[r + 6][tx + dx];
        const int y = y0 + r;
        if (y >= H || x >= W) continue;
        const int c = win[3][4];
        uint32_t lo = 0u, hi = 0u;
        int b = 0;
#pragma unroll
        for (int dy = 0; dy < 7; ++dy) {
#pragma unroll
            for (int dx = 0; dx < 9; ++dx) {
                if (dy == 3 && dx == 4) continue;
                const uint32_t bit = win[dy][dx] < c ? 1u : 0u;
                if (b < 32) lo |= bit << b;
                else hi |= bit << (b - 32);
                ++b;
            }
        }
        out[(size_t)y * W + x] = ((uint64_t)hi << 32) | lo;
    }
}

// ------------------------------------------------------------------ wave helpers
template <int CTRL, int ROWMASK>
__device__ __forceinline__ int dpp_i(int old, int x) {
    return __builtin_amdgcn_update_dpp(old, x, CTRL, ROWMASK, 0xf, false);
}

// Minimum over the 64 lanes, in lane 63: row prefix minima by DPP row
// shifts, then row 0's into row 1 and row 2's into row 3 (row_bcast:15),
// then lane 31's into rows 2 and 3 (row_bcast:31).  Lanes without a source
// take INT_MAX, the identity of the minimum, so that each shift and minimum
// is one v_min_i32_dpp (another fill value costs a move per shift).
constexpr int kNoKey = 0x7fffffff;
__device__ __forceinline__ int wave_min_in63(int x) {
    x = min(x, dpp_i<0x111, 0xf>(kNoKey, x));    // row_shr:1
    x = min(x, dpp_i<0x112, 0xf>(kNoKey, x));    // row_shr:2
    x = min(x, dpp_i<0x114, 0xf>(kNoKey, x));    // row_shr:4
    x = min(x, dpp_i<0x118, 0xf>(kNoKey, x));    // row_shr:8
    x = min(x, dpp_i<0x142, 0xa>(kNoKey, x));    // row_bcast:15 into rows 1 and 3
    x = min(x, dpp_i<0x143, 0xc>(kNoKey, x));    // row_bcast:31 into rows 2 and 3
    return x;
}
__device__ __forceinline__ int wave_min(int x) {
    return __builtin_amdgcn_readlane(wave_min_in63(x), 63);
}

// lane l receives lane l-1's x (lane 0 receives INT_MAX), and lane l+1's
// (lane 63 INT_MAX).  The path step takes them only in a minimum with the
// other neighbour, which is a path cost, so INT_MAX never survives to the
// addition of P1; as the identity of the minimum it lets the shift fold into
// a v_min_i32_dpp.
__device__ __forceinline__ int from_below(int x) { return dpp_i<0x138, 0xf>(0x7fffffff, x); }  // wave_shr:1
__device__ __forceinline__ int from_above(int x) { return dpp_i<0x130, 0xf>(0x7fffffff, x); }  // wave_shl:1

__device__ __forceinline__ int popc64(uint64_t v) {
    return __builtin_popcount((uint32_t)v) + __builtin_popcount((uint32_t)(v >> 32));
}

// DPL consecutive uint16 of S at element offset e (e a multiple of DPL).
// The same DPL values as loaded words (one uint16 zero-extended for DPL 1, a
// dword for 2, two for 4), unpacked only where they are used: a load whose
// value is unpacked at once is waited for at once.
template <int DPL>
using SWord = std::conditional_t<DPL == 4, uint2, uint32_t>;
template <int DPL>
__device__ __forceinline__ SWord<DPL> load_s_word(const uint16_t* S, size_t e) {
    if constexpr (DPL == 1) {
        return (uint32_t)S[e];
    } else if constexpr (DPL == 2) {
        return *reinterpret_cast<const uint32_t*>(S + e);
    } else {
        return *reinterpret_cast<const uint2*>(S + e);
    }
}
template <int DPL>
__device__ __forceinline__ void unpack_s(SWord<DPL> w, int (&v)[DPL]) {
    if constexpr (DPL == 1) {
        v[0] = (int)w;
    } else if constexpr (DPL == 2) {
        v[0] = (int)(w & 0xffffu);
        v[1] = (int)(w >> 16);
    } else {
        v[0] = (int)(w.x & 0xffffu);
        v[1] = (int)(w.x >> 16);
        v[2] = (int)(w.y & 0xffffu);
        v[3] = (int)(w.y >> 16);
    }
}
template <int DPL>
__device__ __forceinline__ void store_s(uint16_t* S, size_t e, const int (&v)[DPL]) {
    if constexpr (DPL == 1) {
        S[e] = (uint16_t)v[0];
    } else if constexpr (DPL == 2) {
        *reinterpret_cast<uint32_t*>(S + e) = (uint32_t)v[0] | ((uint32_t)v[1] << 16);
    } else {
        *reinterpret_cast<uint2*>(S + e) =
            make_uint2((uint32_t)v[0] | ((uint32_t)v[1] << 16), (uint32_t)v[2] | ((uint32_t)v[3] << 16));
    }
}

enum { kFirst = 0, kAdd = 1, kFinal = 2 };

// A bijection of [0, n): block b, the (b / 8)-th block dispatched to XCD
// b mod 8, becomes the (b / 8)-th of that XCD's contiguous range (XCD x
// holds n / 8 blocks, one more if x < n mod 8).
__device__ __forceinline__ int xcd_contiguous(int b, int n) {
    const int x = b & 7, j = b >> 3, q = n >> 3, r = n & 7;
    return x * q + min(x, r) + j;
}


// One path line per wave (a workgroup of one wave).  DIR: 0 left to right,
// 1 right to left, 2 top to bottom, 3 bottom to top.  MODE: kFirst writes S,
// kAdd adds to it, kFinal (left to right only) selects and checks.
// LDS hand-off between the waves of a workgroup: this wave's LDS writes
// have completed before the barrier, and its global loads in flight (later
// steps' operands) are not waited for, as a full fence would.
__device__ __forceinline__ void lds_barrier() {
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_waitcnt(0xc07f);               // lgkmcnt(0)
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
}

// G waves per workgroup (G > 1: column passes only) take G neighbouring
// path lines, one each, and share the right-view census words through LDS.
template <int DPL, int DIR, int MODE, int G = 1>
__global__ __launch_bounds__(64 * G) void path_kernel(PathArgs a) {
    static_assert(MODE != kFinal || DIR == 0, "the final pass runs left to right");
    static_assert(G == 1 || DIR >= 2, "shared census words: column passes");
    extern __shared__ uint32_t lds[];                  // kFinal: keyR[W], then dL[W] (int16)
    constexpr bool HORZ = DIR <= 1;
    constexpr bool STG = G > 1;
    // along a row each step's right-view words are the previous step's moved
    // by one disparity (SLIDE); the final pass reads its wave-uniform words by
    // buffer loads (VLOAD): scalar loads share their wait counter with the
    // pass's LDS atomics, so every wait for one would wait for those too
    constexpr bool SLIDE = HORZ;
    constexpr bool VLOAD = MODE == kFinal;
    const int lane = threadIdx.x & 63;
    const int wv = (G == 1) ? 0 : __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int W = a.W, H = a.H, D = a.D;
    const int lines = HORZ ? H : W;
    const int groups = (lines + G - 1) / G;            // workgroups per frame
    // Workgroups go to the eight XCDs in turn; the launch's blocks are
    // renumbered so that each XCD takes a contiguous range of path lines:
    // neighbouring columns read nearly the same right-view census words
    // every step, and only on one XCD do they share its L2.
    const int bid = xcd_contiguous((int)blockIdx.x, (int)gridDim.x);
    const int f = bid / groups, grp = bid - f * groups;
    // a wave past the last line (G not dividing the lines) repeats the last
    // line with its stores off, so that it still takes part in the barriers
    const bool line_ok = grp * G + wv < lines;
    const int line = min(grp * G + wv, lines - 1);
    const size_t fo = (size_t)f * (size_t)W * (size_t)H;
    const uint64_t* __restrict__ cl = a.cl + fo;
    const uint64_t* __restrict__ cr = a.cr + fo;
    uint16_t* __restrict__ S = a.S + fo * (size_t)D;
    const int steps = HORZ ? W : H;
    const int d0 = lane * DPL;
    const int P1 = a.P1, P2 = a.P2;

    uint32_t* keyR = lds;
    int16_t* dLrow = reinterpret_cast<int16_t*>(lds + (MODE == kFinal ? W : 0));
    if constexpr (MODE == kFinal) {
        for (int x = lane; x < W; x += 64) keyR[x] = 0xffffffffu;
        __syncthreads();
    }

    // pixel of step s
    auto pixel = [&](int s, int& y, int& x) {
        if constexpr (DIR == 0) { y = line; x = s; }
        else if constexpr (DIR == 1) { y = line; x = W - 1 - s; }
        else if constexpr (DIR == 2) { y = s; x = line; }
        else { y = H - 1 - s; x = line; }
    };
    // the census operands of step s; a right-view column left of the image
    // (x - d < 0, whose cost is kCostOut) loads column 0 instead, so that no
    // load sits in a branch (a branch makes the loads of later steps wait)
    auto load_ops = [&](int s, uint64_t& clv, uint64_t (&crv)[DPL]) {
        int y, x;
        pixel(s, y, x);
        clv = cl[(size_t)y * W + x];
#pragma unroll
        for (int i = 0; i < DPL; ++i) crv[i] = cr[(size_t)y * W + max(x - (d0 + i), 0)];
    };

    // Every step's loads (census operands and, after the first pass, the
    // summed costs of its pixel) are issued kAhead steps before the step
    // runs: a wave's step chain is short, so only loads in flight well ahead
    // keep enough bytes moving.  The step loop is unrolled by kAhead so that
    // the ring of loaded values stays in registers.
    // (4: 17.2 ms per 64 pairs of 1024x440, 128 disparities, against 20.7 ms
    // loading a step ahead; 8 steps ahead gained 1 % more for twice the ring)
    constexpr int kAhead = 4;
    uint64_t rcl[kAhead], rcr[kAhead][DPL], rin[SLIDE ? kAhead : 1];
    uint64_t win[DPL];
    SWord<DPL> rsv[kAhead];
    const bool live = d0 < D && line_ok;
    // element of S a step loads: lanes past the disparity range (whose
    // values are never used) load the pixel's last DPL entries
    const int d0l = min(d0, D - DPL);
    auto s_index = [&](int s) {
        int y, x;
        pixel(s, y, x);
        return ((size_t)y * W + x) * (size_t)D + (size_t)d0l;
    };
    // SLIDE: the window of right-view words (lane l, word i: disparity
    // DPL l + i) moves by one lane after each step and takes in one word at
    // its edge lane, so that a step loads two wave-uniform words (the left
    // view's and the entering one) instead of DPL per lane
    const auto clr = make_rsrc(cl, (uint32_t)((size_t)W * H * 8));
    const auto crr = make_rsrc(cr, (uint32_t)((size_t)W * H * 8));
    // word e of a census map through its buffer resource (two dwords)
    auto word_v = [&](__amdgpu_buffer_rsrc_t r, int e) -> uint64_t {
        const uint32_t lo = __builtin_bit_cast(uint32_t, buf_load_b(r, (uint32_t)e * 8u, 0u));
        const uint32_t hi = __builtin_bit_cast(uint32_t, buf_load_b(r, (uint32_t)e * 8u + 4u, 0u));
        return ((uint64_t)hi << 32) | lo;
    };
    auto left_word = [&](int s) -> uint64_t {
        int y, x;
        pixel(s, y, x);
        if constexpr (VLOAD) return word_v(clr, y * W + x);
        else return cl[(size_t)y * W + x];
    };
    // the word that enters the window for step s: disparity 0 moving right,
    // the window's last disparity moving left (column 0 past the image's
    // left edge, as in load_ops)
    auto entering = [&](int s) -> uint64_t {
        int y, x;
        pixel(s, y, x);
        const int xr = (DIR == 0) ? x : max(x - (64 * DPL - 1), 0);
        if constexpr (VLOAD) return word_v(crr, y * W + xr);
        else return cr[(size_t)y * W + xr];
    };
    // the window of the next step, with its entering word e: moving right
    // lane l takes lane l-1's last word (wave_shr:1) and lane 0 takes e;
    // moving left lane l takes lane l+1's first word (wave_shl:1) and lane
    // 63 takes e
    auto slide = [&](uint64_t e) {
        constexpr int C = DIR == 0 ? 0x138 : 0x130;
        const uint64_t v = (DIR == 0) ? win[DPL - 1] : win[0];
        const int lo = dpp_i<C, 0xf>((int)(uint32_t)e, (int)(uint32_t)v);
        const int hi = dpp_i<C, 0xf>((int)(uint32_t)(e >> 32), (int)(uint32_t)(v >> 32));
        const uint64_t in = ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo;
        if constexpr (DIR == 0) {
#pragma unroll
            for (int i = DPL - 1; i > 0; --i) win[i] = win[i - 1];
            win[0] = in;
        } else {
#pragma unroll
            for (int i = 0; i < DPL - 1; ++i) win[i] = win[i + 1];
            win[DPL - 1] = in;
        }
    };
    if constexpr (SLIDE) {
        uint64_t c0;
        load_ops(0, c0, win);
    }
#pragma unroll
    for (int u = 0; u < kAhead; ++u) {
        const int sa = min(u, steps - 1);
        if constexpr (SLIDE) {
            rcl[u] = left_word(sa);
            rin[u] = entering(sa);
        } else if constexpr (STG) {
            int y, x;
            pixel(sa, y, x);
            rcl[u] = cl[(size_t)y * W + x];
        } else {
            load_ops(sa, rcl[u], rcr[u]);
        }
        if constexpr (MODE != kFirst) rsv[u] = load_s_word<DPL>(S, s_index(sa));
    }
    // STG: the right-view words of a group of kAhead rows for all G lines
    // (word j of a row: column x0 - 64 DPL + 1 + j, clamped to the image),
    // loaded by the whole workgroup a group ahead into registers, written to
    // one of two LDS buffers at the group's start and read there by each
    // lane (its words j = wv + 64 DPL - 1 - d)
    constexpr int NSW = 64 * DPL + G - 1;
    constexpr int NPT = STG ? (kAhead * NSW + 64 * G - 1) / (64 * G) : 1;
    // (one word past the rows takes the stores of idle threads: no branch)
    __shared__ uint64_t cst[STG ? 2 : 1][STG ? kAhead * NSW + 1 : 1];
    uint64_t cpre[NPT];
    const int x0 = grp * G;
    auto stage_load = [&](int s0) {
#pragma unroll
        for (int k = 0; k < NPT; ++k) {
            const int idx = (int)threadIdx.x + k * 64 * G;
            const int r = min(idx / NSW, kAhead - 1), j = idx - (idx / NSW) * NSW;
            int y, x;
            pixel(min(s0 + r, steps - 1), y, x);
            cpre[k] = cr[(size_t)y * W + min(max(x0 - 64 * DPL + 1 + j, 0), W - 1)];
        }
    };
    auto stage_store = [&](int buf) {
#pragma unroll
        for (int k = 0; k < NPT; ++k)
            cst[buf][min((int)threadIdx.x + k * 64 * G, kAhead * NSW)] = cpre[k];
    };
    auto stage_ops = [&](int buf, int u, uint64_t (&crc)[DPL]) {
#pragma unroll
        for (int i = 0; i < DPL; ++i) crc[i] = cst[buf][u * NSW + wv + 64 * DPL - 1 - (d0 + i)];
    };
    if constexpr (STG) {
        stage_load(0);
        stage_store(0);
        lds_barrier();
        stage_load(kAhead);
    }

    int Lp[DPL];
    int M = 0;
    // one step of the path at pixel step s, from its loaded operands
    auto step = [&](const int s, const uint64_t clc, const uint64_t (&crc)[DPL],
                    const SWord<DPL> sw) {
        int y, x;
        pixel(s, y, x);
        int L[DPL];
        if (s == 0) {
#pragma unroll
            for (int i = 0; i < DPL; ++i) {
                const int d = d0 + i;
                const int c = (x - d >= 0) ? popc64(clc ^ crc[i]) : kCostOut;
                L[i] = d < D ? c : kBig;
            }
        } else {
            const int below = from_below(Lp[DPL - 1]);   // L(d0 - 1)
            const int above = from_above(Lp[0]);         // L(d0 + DPL)
            const int jump = M + P2;
#pragma unroll
            for (int i = 0; i < DPL; ++i) {
                const int d = d0 + i;
                const int lo = i > 0 ? Lp[i - 1] : below;
                const int hi = i + 1 < DPL ? Lp[i + 1] : above;
                const int t = min(min(Lp[i], min(lo, hi) + P1), jump);
                const int c = (x - d >= 0) ? popc64(clc ^ crc[i]) : kCostOut;
                L[i] = d < D ? c + t - M : kBig;
            }
        }
        int m = L[0];
#pragma unroll
        for (int i = 1; i < DPL; ++i) m = min(m, L[i]);
        M = wave_min(m);
#pragma unroll
        for (int i = 0; i < DPL; ++i) Lp[i] = L[i];

        const size_t e = ((size_t)y * W + x) * (size_t)D + (size_t)d0;
        if constexpr (MODE == kFirst) {
            if (live) store_s<DPL>(S, e, L);
        } else if constexpr (MODE == kAdd) {
            if (live) {
                int v[DPL];
                unpack_s<DPL>(sw, v);
#pragma unroll
                for (int i = 0; i < DPL; ++i) v[i] += L[i];
                store_s<DPL>(S, e, v);
            }
        } else {
            // final summed costs of pixel (y, x): select d_L and offer every
            // d to the right view's column x - d
            int key = kNoKey;
            if (live) {
                int sv[DPL];
                unpack_s<DPL>(sw, sv);
#pragma unroll
                for (int i = 0; i < DPL; ++i) {
                    const int d = d0 + i;
                    const int k = ((sv[i] + L[i]) << 8) | d;
                    key = min(key, k);
                    if (x - d >= 0) atomicMin(&keyR[x - d], (uint32_t)k);
                }
            }
            // lanes without a key hold kNoKey; selection keys stay below 2^23
            const int kmin = wave_min_in63(key);
            if (lane == 63) dLrow[x] = (int16_t)(kmin & 0xff);
        }
    };
    // whole groups of kAhead steps, each step issuing the loads of the step
    // kAhead later (past the line's end the last step is loaded again,
    // unused: a branch here would make each ring slot a merge of two values)
    const int full = steps - steps % kAhead;
    for (int s0 = 0; s0 < full; s0 += kAhead) {
        const int buf = (s0 / kAhead) & 1;
#pragma unroll
        for (int u = 0; u < kAhead; ++u) {
            const int s = s0 + u;
            const uint64_t clc = rcl[u];
            uint64_t crc[DPL];
            if constexpr (STG) {
                stage_ops(buf, u, crc);
            } else if constexpr (SLIDE) {
#pragma unroll
                for (int i = 0; i < DPL; ++i) crc[i] = win[i];
            } else {
#pragma unroll
                for (int i = 0; i < DPL; ++i) crc[i] = rcr[u][i];
            }
            const SWord<DPL> sw = rsv[u];
            // SLIDE: the entering word of step s+1 (its slot is reloaded there)
            const uint64_t en = rin[SLIDE ? (u + 1) % kAhead : 0];
            const int sa = min(s + kAhead, steps - 1);
            if constexpr (SLIDE) {
                rcl[u] = left_word(sa);
                rin[u] = entering(sa);
            } else if constexpr (STG) {
                int y, x;
                pixel(sa, y, x);
                rcl[u] = cl[(size_t)y * W + x];
            } else {
                load_ops(sa, rcl[u], rcr[u]);
            }
            if constexpr (MODE != kFirst) rsv[u] = load_s_word<DPL>(S, s_index(sa));
            step(s, clc, crc, sw);
            if constexpr (SLIDE) slide(en);
        }
        if constexpr (STG) {
            // the next group's words into the other buffer (whose last
            // readers passed the previous barrier), then the group after
            stage_store(buf ^ 1);
            lds_barrier();
            stage_load(s0 + 2 * kAhead);
        }
    }
    // the last steps % kAhead steps, already loaded
#pragma unroll
    for (int u = 0; u < kAhead - 1; ++u) {
        if (full + u < steps) {
            if constexpr (STG) {
                uint64_t crc[DPL];
                stage_ops((full / kAhead) & 1, u, crc);
                step(full + u, rcl[u], crc, rsv[u]);
            } else if constexpr (SLIDE) {
                step(full + u, rcl[u], win, rsv[u]);
                slide(rin[u + 1]);
            } else {
                step(full + u, rcl[u], rcr[u], rsv[u]);
            }
        }
    }
    if constexpr (MODE == kFinal) {
        __syncthreads();
        float* out = a.disp + fo + (size_t)line * W;
        for (int x = lane; x < W; x += 64) {
            const int d = dLrow[x];
            float v = -1.0f;
            if (x - d >= 0) {
                const int e = (int)(keyR[x - d] & 0xffu);
                if (abs(d - e) <= 1) v = (float)d;
            }
            out[x] = v;
        }
    }
}

// columns per workgroup of the column passes (64 pairs 1024x440, 128
// disparities: 16.7 ms per stage with one column per workgroup, 16.5 / 15.7 /
// 15.3 / 15.0 ms with 2 / 4 / 8 / 16)
constexpr int kColumnWaves = 16;

template <int DPL>
hipError_t launch_paths(const PathArgs& a, int frames, hipStream_t st) {
    // the column passes take kColumnWaves columns per workgroup
    const unsigned rows = (unsigned)(frames * a.H);
    const unsigned cgroups = (unsigned)(frames * ((a.W + kColumnWaves - 1) / kColumnWaves));
    hipLaunchKernelGGL((path_kernel<DPL, 2, kFirst, kColumnWaves>), dim3(cgroups),
                       dim3(64 * kColumnWaves), 0, st, a);
    hipLaunchKernelGGL((path_kernel<DPL, 3, kAdd, kColumnWaves>), dim3(cgroups),
                       dim3(64 * kColumnWaves), 0, st, a);
    hipLaunchKernelGGL((path_kernel<DPL, 1, kAdd>), dim3(rows), dim3(64), 0, st, a);
    const size_t lds = (size_t)a.W * sizeof(uint32_t) + (size_t)a.W * sizeof(int16_t);
    hipLaunchKernelGGL((path_kernel<DPL, 0, kFinal>), dim3(rows), dim3(64), lds, st, a);
    return hipGetLastError();
}

}  // namespace

int dpl_of(int D) { return D <= 64 ? 1 : (D <= 128 ? 2 : 4); }

hipError_t launch_sgm(const uint8_t* left, const uint8_t* right, int W, int H, int frames,
                      const SgmWorkspace& ws, int D, int P1, int P2, float* disp, hipStream_t st) {
    dim3 grid((unsigned)((W + kTileW - 1) / kTileW), (unsigned)((H + kTileH - 1) / kTileH),
              (unsigned)(2 * frames));
    hipLaunchKernelGGL(census_kernel, grid, dim3(256), 0, st, left, right, W, H, ws.cl, ws.cr);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    PathArgs a{ws.cl, ws.cr, ws.S, disp, W, H, D, P1, P2};
    switch (dpl_of(D)) {
        case 1: return launch_paths<1>(a, frames, st);
        case 2: return launch_paths<2>(a, frames, st);
        default: return launch_paths<4>(a, frames, st);
    }
}

}  // namespace stx::sgm

// ------------------------------------------------------------------ C ABI
struct stixels_sgm {
    stixels_sgm_params p{};
    stx::sgm::SgmWorkspace ws{};
    size_t bytes = 0;
    int last_W = 0, last_H = 0, device = 0;
    std::string err;
};

namespace {

int sgm_fail(stixels_sgm* m, int code, const std::string& msg) {
    if (m) m->err = msg;
    return code;
}

thread_local std::string g_sgm_create_error;

}  // namespace

extern "C" {

int stixels_sgm_create(const stixels_sgm_params* params, stixels_sgm** out) {
    if (!params || !out) return STIXELS_E_INVALID_ARG;
    *out = nullptr;
    const stixels_sgm_params& p = *params;
    const char* why = nullptr;
    if (p.max_width < 1 || p.max_height < 1) why = "max_width and max_height must be >= 1";
    else if (p.max_disparity < 4 || p.max_disparity > 256 || p.max_disparity % 4 != 0)
        why = "max_disparity must be a multiple of 4 in 4..256";
    else if (p.p1 < 0 || p.p2 < p.p1 || p.p2 > 1000) why = "penalties need 0 <= p1 <= p2 <= 1000";
    else if (p.paths != 4) why = "paths must be 4 (the four axis directions)";
    else if (p.max_frames < 1) why = "max_frames must be >= 1";
    else if (p.max_width > 8192) why = "max_width must be <= 8192 (a row's selection state in LDS)";
    if (why) {
        g_sgm_create_error = why;
        return STIXELS_E_INVALID_ARG;
    }
    stixels_sgm* m = new (std::nothrow) stixels_sgm;
    if (!m) return STIXELS_E_NOMEM;
    m->p = p;
    (void)hipGetDevice(&m->device);
    const size_t n = (size_t)p.max_frames * (size_t)p.max_width * (size_t)p.max_height;
    const size_t nd = n * (size_t)p.max_disparity;
    bool ok = hipMalloc(reinterpret_cast<void**>(&m->ws.cl), n * sizeof(uint64_t)) == hipSuccess &&
              hipMalloc(reinterpret_cast<void**>(&m->ws.cr), n * sizeof(uint64_t)) == hipSuccess &&
              hipMalloc(reinterpret_cast<void**>(&m->ws.S), nd * sizeof(uint16_t)) == hipSuccess;
    m->bytes = 2 * n * sizeof(uint64_t) + nd * sizeof(uint16_t);
    if (!ok) {
        (void)hipFree(m->ws.cl);
        (void)hipFree(m->ws.cr);
        (void)hipFree(m->ws.S);
        delete m;
        g_sgm_create_error = "hipMalloc of the matching workspace failed";
        return STIXELS_E_NOMEM;
    }
    *out = m;
    return STIXELS_OK;
}

int stixels_sgm_destroy(stixels_sgm* m) {
    if (!m) return STIXELS_OK;
    (void)hipFree(m->ws.cl);
    (void)hipFree(m->ws.cr);
    (void)hipFree(m->ws.S);
    delete m;
    return STIXELS_OK;
}

const char* stixels_sgm_last_error(const stixels_sgm* m) {
    return m ? m->err.c_str() : g_sgm_create_error.c_str();
}

int stixels_sgm_device_bytes(const stixels_sgm* m, size_t* bytes) {
    if (!m || !bytes) return STIXELS_E_INVALID_ARG;
    *bytes = m->bytes;
    return STIXELS_OK;
}

int stixels_sgm_compute(stixels_sgm* m, const uint8_t* d_left, const uint8_t* d_right,
                        int32_t width, int32_t height, int32_t frames, void* stream,
                        float* d_disparity) {
    if (!m) return STIXELS_E_INVALID_ARG;
    if (!d_left || !d_right || !d_disparity)
        return sgm_fail(m, STIXELS_E_INVALID_ARG, "null image or disparity pointer");
    if (width < 1 || width > m->p.max_width || height < 1 || height > m->p.max_height)
        return sgm_fail(m, STIXELS_E_INVALID_ARG, "width or height outside the handle's maximum");
    if (frames < 1 || frames > m->p.max_frames)
        return sgm_fail(m, STIXELS_E_INVALID_ARG, "frames outside [1, max_frames]");
    const hipError_t e =
        stx::sgm::launch_sgm(d_left, d_right, width, height, frames, m->ws, m->p.max_disparity,
                             m->p.p1, m->p.p2, d_disparity, static_cast<hipStream_t>(stream));
    if (e != hipSuccess)
        return sgm_fail(m, STIXELS_E_HIP, std::string("kernel launch failed: ") + hipGetErrorString(e));
    m->last_W = width;
    m->last_H = height;
    return STIXELS_OK;
}

int stixels_sgm_debug(const stixels_sgm* m, int32_t which, void* host_dst, size_t bytes) {
    if (!m || !host_dst || which < 0 || which > 2) return STIXELS_E_INVALID_ARG;
    const size_t n = (size_t)m->last_W * (size_t)m->last_H;
    if (n == 0) return STIXELS_E_INVALID_ARG;
    const void* src = which == 0 ? (const void*)m->ws.cl
                                 : (which == 1 ? (const void*)m->ws.cr : (const void*)m->ws.S);
    const size_t need = which == 2 ? n * (size_t)m->p.max_disparity * sizeof(uint16_t)
                                   : n * sizeof(uint64_t);
    if (bytes < need) return STIXELS_E_INVALID_ARG;
    if (hipDeviceSynchronize() != hipSuccess ||
        hipMemcpy(host_dst, src, need, hipMemcpyDeviceToHost) != hipSuccess)
        return STIXELS_E_HIP;
    return STIXELS_OK;
}

int stixels_compute_stereo(stixels_handle* h, stixels_sgm* m, const uint8_t* d_left,
                           const uint8_t* d_right, int32_t width, int32_t height, void* stream,
                           float* d_disparity, const stixels_output* out) {
    if (!h || !m) return STIXELS_E_INVALID_ARG;
    if (m->p.max_disparity != h->p.max_disparity || h->p.subpixel_log2 != 0) {
        h->err = "the matching handle's max_disparity must equal the stixel handle's (whole pixels)";
        return STIXELS_E_INVALID_ARG;
    }
    int rc = stixels_sgm_compute(m, d_left, d_right, width, height, 1, stream, d_disparity);
    if (rc != STIXELS_OK) {
        h->err = m->err;
        return rc;
    }
    return stixels_compute(h, d_disparity, width, height, stream, out);
}

}  // extern "C"
