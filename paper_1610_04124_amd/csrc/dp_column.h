// dp_column.h -- the Eq. 5-6 recurrence and backtracking for one column, run
// by W wave64s (W = 1, 2 or 4).
//
// Work distribution (gfx950): the rows are cut into 64-row slots s < S; slot
// s belongs to wave s mod W (interleaved, so that the waves keep an even
// share of the rows still open as the recurrence advances), and lane l of
// that wave owns row k = 64 s + l, with its running minimum OB^k, the mean of
// the best object stixel ending at k and the prefix values at k+1 in VGPRs.
// The recurrence is evaluated in push form: once row j is final (all
// candidates with a cut at b <= j have been seen), its values are read from
// the owning lane with v_readlane (and, with W > 1, passed to the other
// waves through LDS behind one barrier per step) and every lane folds the
// candidates that start at b = j+1 into its rows k > j.  There is no
// cross-lane reduction per step, unlike the one-thread-per-k CTA of
// Sec. 4.3.
//
// The index table of Sec. 3.3 is not stored.  Because every cost is exact on
// the grid, backtracking recovers each link by recomputing the candidates of
// a row and taking the first one equal to the row's minimum, in the order of
// Eq. 6: the bottom-stixel candidate, then cut positions b ascending, then
// predecessor classes object, ground, sky.  This is the same choice as a
// first-minimum index table.
#pragma once

#include <type_traits>

#include "internal.h"

namespace stx {

// f(std::integral_constant<int, I>) for I = B .. E-1, in order.
template <int B, int E, class F>
__device__ __forceinline__ void static_for(F&& f) {
    if constexpr (B < E) {
        f(std::integral_constant<int, B>{});
        static_for<B + 1, E>(f);
    }
}

struct ColumnIn {
    const float* PG;        // [H+1] ground cost prefix
    const float* PS;        // [H+1] sky cost prefix
    const float* PA;        // [H+1] prefix of 2*q+1 over valid pixels
    const float* PN2;       // [H+1] prefix of 2 over valid pixels
    const float* PO;        // [fmax-fbase+1][po_stride] object cost prefix, row f-fbase
    int fbase, fmax;        // disparity rows of PO (fbase = 0 if the column has an invalid pixel)
    int po_stride = 0;      // floats from one PO row to the next (0: H+1)
    // banded object prefix table (solve_column with BAND): per 64-row slot t,
    // the first mean band_lo[t] of its band and the float offset band_base[t]
    // of its rows within PO (LDS arrays)
    const int* band_lo = nullptr;
    const int* band_base = nullptr;
    uint32_t po_bytes = 0;  // bytes of the PO table (0: its rows times po_stride)
    // solve_column with RT: rcp(2 n) for n = 0 .. 64 S (LDS), the values
    // v_rcp_f32 gives, read in place of that instruction (which takes about
    // two VALU issue slots)
    const float* rtab = nullptr;
    const int16_t* q;       // [H] reduced disparities of the column (LDS), -1 invalid
    const float* O_df;      // [D][D] object cost, row d (pixel disparity), column f (mean)
    int D;
    const int32_t* fg_hi;   // diving threshold per top-down image row
    const int32_t* fg_lo;   // gravity threshold per top-down image row
    float* rowc;            // [4][H+1] final object, ground, sky cost and best mean (bits) of
                            // every row, for the two-column recurrence only
    const float* S_tab;     // [D] sky cost per pixel disparity (costs off the grid only)
    const float* G_tab;     // [rows][D] ground cost by top-down row (costs off the grid only)
};

// Cut position b of the best stixel of each class ending at every row (the
// index table of Sec. 3.3), kept by the recurrence variant for costs that
// are not on a grid, whose backtracking cannot recover links by exact
// recomputation.
template <int S, bool LINKS>
struct LinkRows {};
template <int S>
struct LinkRows<S, true> {
    int16_t b[3][64 * S];
};

// Per-workgroup LDS of one column (S slots, W waves, QT prior-table entries
// per wave: 64 per disparity chunk).
template <int S, int W, int QT = 256, bool LINKS = false>
struct ColumnLds {
    float qtab[W][QT + 4];  // per wave: prior minus PO[f][b] over the disparity rows (from +4)
    float crow_g[64 * S];   // final GR^k of every row
    float crow_s[64 * S];   // final SK^k
    float crow_o[64 * S];   // final OB^k
    uint8_t crow_f[64 * S]; // mean - fbase of the best object stixel ending at k
    float bc[2][4];         // row j's values for the other waves (double-buffered)
    LinkRows<S, LINKS> lk;  // object, ground, sky links (LINKS only)
};

struct ColumnOut {
    int32_t* count;
    uint32_t* rec;          // capacity records of 3 dwords (stixels_record)
    float* total;
    uint8_t* overflow;
    int cap;
#ifdef STX_PHASE_TIMING
    unsigned long long* t_rec_end = nullptr;   // shader clock when the recurrence ends
#endif
};

// Emitted stixel, kept by lane t (t-th stixel found from the top).
struct RecRegs {
    uint32_t w0, w1;
    float w2;
};

__device__ __forceinline__ void pack_record(int vb, int vt, int cls, int f, float cost,
                                            uint32_t& w0, uint32_t& w1, float& w2) {
    w0 = (uint32_t)(vb & 0xffff) | ((uint32_t)(vt & 0xffff) << 16);
    w1 = (uint32_t)(cls & 0xff) | ((uint32_t)(f & 0xff) << 8);
    w2 = cost;
}

// a[c] for a class index known only at run time, without indexable memory
__device__ __forceinline__ float pick3(float a0, float a1, float a2, int c) {
    return c == 0 ? a0 : (c == 1 ? a1 : a2);
}

// Backtracking of one column (Sec. 3.3, Sec. 4.4) by one wave64: every
// row's final object, ground and sky cost and best object mean are in LDS
// (L.crow_*), its prefix values in the column's tables (in).
// BAND: the column's object prefix table is banded (solve_column), so the
// object data terms are taken from the full prefix row of the stored mean of
// the row's best object stixel, recomputed here (the first optimal candidate
// has that mean).
template <int S, class Lds, bool BAND = false>
__device__ __forceinline__ void backtrack_column(const int H, const int vtop, const Prior P, const ColumnIn& in,
                                 const ColumnOut& out, const Lds& L) {
    const int lane = threadIdx.x & 63;
    const int stride = H + 1;
    const uint32_t stride4 = (uint32_t)stride * 4u;
    const int pstride = in.po_stride ? in.po_stride : stride;
    const int fbase = in.fbase;
    const int nrow = in.fmax - fbase + 1;
    const auto po = make_rsrc(in.PO, (uint32_t)(nrow * pstride) * 4u);
    const auto pgr = make_rsrc(in.PG, stride4);
    const auto psr = make_rsrc(in.PS, stride4);
    const auto par = make_rsrc(in.PA, stride4);
    const auto pnr = make_rsrc(in.PN2, stride4);
    const float eps = P.mean_eps;
    const float INF = inf_f();

    const int ktop = H - 1;
    float total = L.crow_o[ktop];
    int ctop = 0;
    {
        const float g = L.crow_g[ktop], sk = L.crow_s[ktop];
        if (g < total) { total = g; ctop = 1; }
        if (sk < total) { total = sk; ctop = 2; }
    }

    // Walk the links from the top.  direct = false keeps the first 64
    // stixels in lane registers (stixel t in lane t) and only counts the
    // rest; direct = true writes every stixel straight to its bottom-up
    // position (second pass, needed only for more than 64 stixels).
    // BAND: R[s] = full object prefix of mean fr at entry 64 s + lane + 1
    float R[BAND ? S : 1];
    int fr = -1;
    auto prefix_row = [&](int f) {
        const auto odf = make_rsrc(in.O_df, (uint32_t)(in.D * in.D) * 4u);
        float carry = 0.0f;
#pragma unroll
        for (int s = 0; s < S; ++s) {
            const int v = 64 * s + lane;
            // the pixel of row v from the integer prefixes (2q+1 and 2 per valid pixel)
            float o = 0.0f;
            if (v < H) {
                const float n2 = buf_load(pnr, v + 1) - buf_load(pnr, v);
                const float a = buf_load(par, v + 1) - buf_load(par, v);
                if (n2 != 0.0f) o = buf_load(odf, ((int)a >> 1) * in.D + f);
            }
            const float r = wave_inclusive_scan(o) + carry;
            R[s] = r;
            carry = readlane_f(r, 63);
        }
        fr = f;
    };
    auto walk = [&](bool direct, int n_total, RecRegs& rr) -> int {
        int k = ktop, cls = ctop, t = 0;
        float target = total;
        while (true) {
            const float kG = (k <= vtop) ? buf_load(pgr, k + 1) : INF;
            const float kS = buf_load(psr, k + 1);
            const float kA = buf_load(par, k + 1), kN = buf_load(pnr, k + 1);
            const int kk = k + 1;
            int lb = -1, lc = -1, lf = 0;
            float prevC = 0.0f;
            // priors of the three predecessor classes into class cls
            const float tO = pick3(P.trans[0][0], P.trans[0][1], P.trans[0][2], cls);
            const float tG = pick3(P.trans[1][0], P.trans[1][1], P.trans[1][2], cls);
            const float tS = pick3(P.trans[2][0], P.trans[2][1], P.trans[2][2], cls);
            // BAND: the full prefix row of the stored mean of row k's best
            // object stixel, and its entry at k+1
            int fstar = 0;
            float rk = 0.0f;
            if constexpr (BAND) {
                if (cls == 0) {
                    fstar = (int)L.crow_f[k] + fbase;
                    if (fstar != fr) prefix_row(fstar);
#pragma unroll
                    for (int s = 0; s < S; ++s)
                        if (s == (k >> 6)) rk = readlane_f(R[s], k & 63);
                }
            }
            {   // bottom stixel b = 0 (prefix entries at 0 are zero)
                int f0 = 0;
                float d0;
                bool ok = true;
                if (cls == 0) {
                    f0 = rounded_mean(kA, kN, eps);
                    if constexpr (BAND) {
                        d0 = rk;
                        ok = (f0 == fstar);
                    } else {
                        d0 = buf_load(po, (f0 - fbase) * pstride + kk);
                    }
                } else {
                    d0 = (cls == 1) ? kG : kS;
                }
                if (ok && d0 + pick3(P.first[0], P.first[1], P.first[2], cls) == target) {
                    lb = 0;
                    lf = f0;
                }
            }
            // The slots holding predecessor rows p < k go in groups: a group's
            // prefix loads are issued together, then its table gathers, then
            // its candidates are checked in b order (lanes past the row form
            // out-of-range indices, which the buffer bounds checks read as 0).
            constexpr int BG = (S <= 4) ? S : 4;
            const auto fgh = make_rsrc(in.fg_hi, (uint32_t)H * 4u);
            const auto fgl = make_rsrc(in.fg_lo, (uint32_t)H * 4u);
            for (int g0 = 0; g0 < S; g0 += BG) {
                if (lb >= 0 || g0 * 64 >= k) break;
                float pa[BG], pn[BG], dk[BG], db[BG];
                int fv[BG], thi[BG], tlo[BG];
#pragma unroll
                for (int i = 0; i < BG; ++i) {
                    const int s = g0 + i;
                    if (s >= S || s * 64 >= k) break;
                    const int bb = s * 64 + lane + 1;
                    if (cls == 0) {
                        pa[i] = buf_load(par, bb);
                        pn[i] = buf_load(pnr, bb);
                    } else {
                        pa[i] = buf_load((cls == 1) ? pgr : psr, bb);
                    }
                }
                if (cls == 0) {
#pragma unroll
                    for (int i = 0; i < BG; ++i) {
                        const int s = g0 + i;
                        if (s >= S || s * 64 >= k) break;
                        const int p = s * 64 + lane, bb = p + 1;
                        const int f = rounded_mean(kA - pa[i], kN - pn[i], eps);
                        fv[i] = f;
                        if constexpr (BAND) {
                            dk[i] = rk;
                            db[i] = R[s];          // entry p+1 = 64 s + lane + 1
                        } else {
                            dk[i] = buf_load(po, (f - fbase) * pstride + kk);
                            db[i] = buf_load(po, (f - fbase) * pstride + bb);
                        }
                        const int r = (p < k) ? H - 1 - bb : 0;
                        thi[i] = __builtin_bit_cast(int, buf_load(fgh, r));
                        tlo[i] = __builtin_bit_cast(int, buf_load(fgl, r));
                    }
                }
#pragma unroll
                for (int i = 0; i < BG; ++i) {
                    const int s = g0 + i;
                    if (s >= S || s * 64 >= k) break;
                    const int p = s * 64 + lane;     // predecessor row, cut at b = p+1
                    const bool inr = p < k;
                    float data;
                    int f = 0;
                    float pen_o = 0.0f, pen_g = 0.0f;
                    const float mo = L.crow_o[p], mg = L.crow_g[p], ms = L.crow_s[p];   // p < 64 S
                    if (cls == 0) {
                        f = fv[i];
                        data = dk[i] - db[i];
                        pen_o = (f > (int)L.crow_f[p] + fbase + P.tau_ord) ? P.c_ord : 0.0f;
                        pen_g = (f > thi[i]) ? P.c_dive : ((f < tlo[i]) ? P.c_grav : 0.0f);
                    } else {
                        // ground stixels end at or below vtop, so PG[p+1] is finite
                        data = ((cls == 1) ? kG : kS) - pa[i];
                    }
                    const float co = mo + tO + pen_o + data;
                    const float cg = mg + tG + pen_g + data;
                    const float cs = ms + tS + data;
                    // BAND: an object candidate whose mean is not the stored one
                    // is not the first optimal one
                    const bool skip = !inr || (BAND && cls == 0 && f != fstar);
                    const int code = skip ? 3
                                   : (co == target ? 0 : (cg == target ? 1 : (cs == target ? 2 : 3)));
                    const uint64_t m = __ballot(code < 3);
                    if (m) {
                        const int l0 = (int)__builtin_ctzll(m);
                        lb = s * 64 + l0 + 1;
                        lc = readlane_i(code, l0);
                        lf = readlane_i(f, l0);
                        const float pc = (lc == 0) ? mo : ((lc == 1) ? mg : ms);
                        prevC = readlane_f(pc, l0);
                        break;
                    }
                }
            }
            if (lb < 0) return -1;
            const float cost = (lb > 0) ? target - prevC : target;
            const int fout = (cls == 0) ? lf : 0;
            if (!direct) {
                if (lane == t) pack_record(lb, k, cls, fout, cost, rr.w0, rr.w1, rr.w2);
            } else {
                const int pos = n_total - 1 - t;
                if (pos < out.cap && lane == 0) {
                    uint32_t w0, w1;
                    float w2;
                    pack_record(lb, k, cls, fout, cost, w0, w1, w2);
                    out.rec[pos * 3 + 0] = w0;
                    out.rec[pos * 3 + 1] = w1;
                    out.rec[pos * 3 + 2] = __builtin_bit_cast(uint32_t, w2);
                }
            }
            ++t;
            if (lb == 0) break;
            k = lb - 1;
            cls = lc;
            target = prevC;
        }
        return t;
    };

    RecRegs rr{0u, 0u, 0.0f};
    const int n = walk(false, 0, rr);
    if (n < 0) {
        if (lane == 0) {
            *out.count = 0;
            *out.total = total;
            *out.overflow = 255;
        }
        return;
    }
    if (n <= 64) {
        const int pos = n - 1 - lane;
        if (lane < n && pos < out.cap) {
            out.rec[pos * 3 + 0] = rr.w0;
            out.rec[pos * 3 + 1] = rr.w1;
            out.rec[pos * 3 + 2] = __builtin_bit_cast(uint32_t, rr.w2);
        }
    } else {
        RecRegs dummy{0u, 0u, 0.0f};
        walk(true, n, dummy);
    }
    if (lane == 0) {
        *out.count = n < out.cap ? n : out.cap;
        *out.total = total;
        *out.overflow = (uint8_t)(n > out.cap ? 1 : 0);
    }
}

// Backtracking along stored links (Sec. 3.3, Sec. 4.4) by one wave64, for
// the recurrence variant that keeps them (L.lk): the cut position of each
// row's best stixel per class is read, and the predecessor class is the
// first class (object, ground, sky) attaining the minimum the recurrence
// took at that cut, recomputed from the same operands with the same
// operations, hence bit for bit.  On the cost grid a stixel's cost is the
// difference of two row costs (exact); off the grid (P.exact = 0) its data
// term is summed directly over its pixels, recovered from the integer
// prefixes (2q+1 and 2 per valid pixel), so that prefix cancellation does
// not enter the reported cost, and its prior is added from the constants.
template <int S, class Lds>
__device__ __forceinline__ void backtrack_links(const int H, const int vtop, const Prior P, const ColumnIn& in,
                                const ColumnOut& out, const Lds& L) {
    const int lane = threadIdx.x & 63;
    const int fbase = in.fbase;
    const float INF = inf_f();
    const int ktop = H - 1;
    float total = L.crow_o[ktop];
    int ctop = 0;
    {
        const float g = L.crow_g[ktop], sk = L.crow_s[ktop];
        if (g < total) { total = g; ctop = 1; }
        if (sk < total) { total = sk; ctop = 2; }
    }
    // data term of stixel [b, k] of class cls (mean f) as a direct sum
    auto direct = [&](int cls, int b, int k, int f) -> float {
        float acc = 0.0f;
        for (int v0 = b; v0 <= k; v0 += 64) {
            const int v = v0 + lane;
            if (v <= k && in.PN2[v + 1] != in.PN2[v]) {
                const int q = (int)((in.PA[v + 1] - in.PA[v] - 1.0f) * 0.5f);
                acc += (cls == 0) ? in.O_df[q * in.D + f]
                                  : ((cls == 1) ? in.G_tab[(size_t)(H - 1 - v) * in.D + q]
                                                : in.S_tab[q]);
            }
        }
        return readlane_f(wave_inclusive_scan(acc), 63);
    };
    auto walk = [&](bool direct_write, int n_total, RecRegs& rr) -> int {
        int k = ktop, cls = ctop, t = 0;
        float target = total;
        while (true) {
            const int b = (int)L.lk.b[cls][k];
            const int f = (cls == 0) ? (int)L.crow_f[k] + fbase : 0;
            int cp = -1;
            float prevC = 0.0f, prior = pick3(P.first[0], P.first[1], P.first[2], cls);
            if (b > 0) {
                const int p = b - 1;
                const float Co = L.crow_o[p], Cg = L.crow_g[p], Cs = L.crow_s[p];
                float x0, x1, x2, pen0 = 0.0f, pen1 = 0.0f;
                if (cls == 0) {
                    const float Xoo = Co + P.trans[0][0];
                    const bool ord = f > (int)L.crow_f[p] + fbase + P.tau_ord;
                    x0 = ord ? Xoo + P.c_ord : Xoo;
                    pen0 = ord ? P.c_ord : 0.0f;
                    x1 = INF;
                    if (b <= vtop + 1) {          // steps with the ground terms
                        const int r = H - 1 - b;
                        const int thi = in.fg_hi[r], tlo = in.fg_lo[r];
                        const float Xgo = Cg + P.trans[1][0];
                        x1 = (f < tlo) ? Xgo + P.c_grav : Xgo;
                        pen1 = (f < tlo) ? P.c_grav : 0.0f;
                        if (f > thi) {
                            x1 = Xgo + P.c_dive;
                            pen1 = P.c_dive;
                        }
                    }
                    x2 = Cs + P.trans[2][0];
                } else {
                    x0 = Co + pick3(P.trans[0][0], P.trans[0][1], P.trans[0][2], cls);
                    x1 = Cg + pick3(P.trans[1][0], P.trans[1][1], P.trans[1][2], cls);
                    x2 = Cs + pick3(P.trans[2][0], P.trans[2][1], P.trans[2][2], cls);
                }
                const float m = vmin(vmin(x0, x1), x2);
                cp = (x0 == m) ? 0 : ((x1 == m) ? 1 : 2);
                prevC = pick3(Co, Cg, Cs, cp);
                prior = pick3(P.trans[0][cls], P.trans[1][cls], P.trans[2][cls], cp) +
                        ((cp == 0) ? pen0 : ((cp == 1) ? pen1 : 0.0f));
            }
            float cost;
            if (P.exact) {
                cost = (b > 0) ? target - prevC : target;
            } else {
                cost = direct(cls, b, k, f) + prior;
            }
            const int fout = (cls == 0) ? f : 0;
            if (!direct_write) {
                if (lane == t) pack_record(b, k, cls, fout, cost, rr.w0, rr.w1, rr.w2);
            } else {
                const int pos = n_total - 1 - t;
                if (pos < out.cap && lane == 0) {
                    uint32_t w0, w1;
                    float w2;
                    pack_record(b, k, cls, fout, cost, w0, w1, w2);
                    out.rec[pos * 3 + 0] = w0;
                    out.rec[pos * 3 + 1] = w1;
                    out.rec[pos * 3 + 2] = __builtin_bit_cast(uint32_t, w2);
                }
            }
            ++t;
            if (b == 0 || t > H) break;
            k = b - 1;
            cls = cp;
            target = prevC;
        }
        return t;
    };

    RecRegs rr{0u, 0u, 0.0f};
    const int n = walk(false, 0, rr);
    if (n <= 64) {
        const int pos = n - 1 - lane;
        if (lane < n && pos < out.cap) {
            out.rec[pos * 3 + 0] = rr.w0;
            out.rec[pos * 3 + 1] = rr.w1;
            out.rec[pos * 3 + 2] = __builtin_bit_cast(uint32_t, rr.w2);
        }
    } else {
        RecRegs dummy{0u, 0u, 0.0f};
        walk(true, n, dummy);
    }
    if (lane == 0) {
        *out.count = n < out.cap ? n : out.cap;
        *out.total = total;
        *out.overflow = (uint8_t)(n > out.cap ? 1 : 0);
    }
}

// S: 64-row slots (h <= 64 S); NCH: 64-entry chunks of disparity rows
// (d_range <= 64 NCH); W: waves per column (the workgroup is 64 W lanes, all
// of which call this function).  POL: the recurrence gathers the object
// prefix table from po_lds, an LDS copy of in.PO (the backtracking still
// reads in.PO).  BLOCKS: short columns read their steps' wave-uniform
// values a slot at a time (right for many waves per SIMD, which hide the
// load at each slot boundary; a column alone on its SIMD keeps the per-step
// prefetch).  LINKS: also keep the cut position of every row's best stixel
// per class (one select per candidate) and backtrack along those links, for
// costs off the grid.  BAND (costs on the grid): the object
// prefix table holds, per 64-row slot t, only the rows of the means that a
// stixel ending in the slot can take, [band_lo[t], band_hi[t]], after one row
// of +inf: row r of slot t is mean band_lo[t] + r - 1, entry 64 t + l + 1 at
// float l.  The mean index of a candidate is then relative to its slot's
// band; a stixel without valid pixels (mean 0, index 0) reads the +inf row
// and is folded separately with its exact cost.  RT: the reciprocal 1/(2n)
// of a candidate's rounded mean comes from in.rtab (an LDS table of the
// values v_rcp_f32 gives, so every mean is the same), the row counts are
// kept as byte offsets n * 4 into it: one LDS read replaces a subtraction
// and a v_rcp_f32, which takes about two VALU issue slots.  On return the
// results are written.
template <int S, int NCH, int W, bool POL = false, bool BLOCKS = true, bool LINKS = false,
          bool BAND = false, bool RT = false>
__device__ __forceinline__ void solve_column(const int H, const int vtop, const Prior P, const ColumnIn& in,
                             const ColumnOut& out, ColumnLds<S, W, 64 * NCH, LINKS>& L,
                             const float* po_lds = nullptr) {
    static_assert(W == 1 || W == 2 || W == 4, "waves per column");
    constexpr int SW = (S + W - 1) / W;              // slots per wave
    const int lane = threadIdx.x & 63;
    const int wave = (W == 1) ? 0 : __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int stride = H + 1;
    const uint32_t stride4 = (uint32_t)stride * 4u;
    const uint32_t pstride4 = (uint32_t)(in.po_stride ? in.po_stride : stride) * 4u;
    const int fbase = in.fbase, fmax = in.fmax;
    const int nrow = fmax - fbase + 1;               // <= d_range <= 64 * NCH
    const auto po = make_rsrc(in.PO, in.po_bytes ? in.po_bytes : (uint32_t)nrow * pstride4);
    // object prefix entry at byte offset `off` of the column's table; the
    // LDS copy clamps the offset to the table (rows past the column's height
    // form arbitrary offsets), the buffer resource reads 0 past its end
    const uint32_t po_last = (uint32_t)nrow * pstride4 - 4u;
    auto po_at = [&](uint32_t off, uint32_t soff) -> float {
        if constexpr (POL) {
            return po_lds[__builtin_elementwise_min(off + soff, po_last) >> 2];
        } else {
            return buf_load_b(po, off, soff);
        }
    };
    const float eps = P.mean_eps;
    using NT = std::conditional_t<RT, int, float>;
    const float cmean = eps - (float)fbase;          // mean_index gives f - fbase
    const float INF = inf_f();
    // rounded mean index from the prefix differences of the numerator and
    // of the row count (2 n, or with RT its byte offset into the reciprocal
    // table), and a row count read from a lane
    const float* const rtab = in.rtab;
    auto mean_of = [&](float a, NT nd, float c) -> int {
        if constexpr (RT) {
            const float r =
                *reinterpret_cast<const float*>(reinterpret_cast<const char*>(rtab) + nd);
            return cvt_i32_nan0(__builtin_fmaf(a, r, c));
        } else {
            return mean_index(a, nd, c);
        }
    };
    auto readlane_n = [](NT v, int l) -> NT {
        if constexpr (RT) return readlane_i(v, l);
        else return readlane_f(v, l);
    };
    const uint32_t lane4 = (uint32_t)(lane + 1) * 4u;   // byte offset of row k+1 within a slot
    const auto pgr = make_rsrc(in.PG, stride4);
    const auto psr = make_rsrc(in.PS, stride4);
    float* const qtab = L.qtab[wave] + 4;
    static_assert(!BAND || !LINKS, "banded tables: costs on the grid");
    // BAND, per slot t: the mean-index constant of its band (index = mean -
    // band_lo[t] + 1), its rows' byte offset within PO and the byte offset,
    // within the prior table, of index 0 (mean band_lo[t] - 1)
    float bcm[BAND ? SW : 1];
    uint32_t bsb[BAND ? SW : 1];
    int bqo[BAND ? SW : 1];

    // local slot t of this wave is global slot t W + wave
    // prefix values at k+1: mean numerator and 2 n (RT: n * 4, a byte offset
    // into the reciprocal table)
    float eA[SW];
    NT eN[SW];
    float mO[SW];                       // OB^k so far
    int fO[SW];                         // mean (- fbase) of the best object stixel ending at k
    int bO[LINKS ? SW : 1];             // its cut position (LINKS)

    // Slots past the column's height (a shorter frame in a batch sized for
    // taller ones, or the last slot of a wave when W does not divide S) are
    // padding: their rows are never read.
    const int nslots = (H + 63) >> 6;

    if constexpr (BAND) {
#pragma unroll
        for (int t = 0; t < SW; ++t) {
            const int sg = t * W + wave;                // global slot
            const int lo = __builtin_amdgcn_readfirstlane(in.band_lo[sg]);
            bcm[t] = P.mean_eps - (float)(lo - 1);
            bsb[t] = (uint32_t)__builtin_amdgcn_readfirstlane(in.band_base[sg]) * 4u;
            bqo[t] = (lo - 1 - fbase) * 4;
        }
    }
    const uint32_t lane4b = (uint32_t)lane * 4u;     // entry 64 t + lane + 1 of a band row

    // Bottom-stixel candidates (b = 0): data(0, k) + F[c] + beta.
#pragma unroll
    for (int t = 0; t < SW; ++t) {
        const int s = t * W + wave;
        if constexpr (LINKS) bO[t] = 0;
        if (s >= nslots) {
            mO[t] = INF;
            eA[t] = 0.0f;
            eN[t] = 0;
            fO[t] = 0;
            continue;
        }
        const int k = s * 64 + lane;
        const int kk = min(k + 1, H);
        eA[t] = in.PA[kk];
        if constexpr (RT) {
            eN[t] = (int)in.PN2[kk] * 2;
        } else {
            eN[t] = in.PN2[kk];
        }
        if constexpr (BAND) {
            // mean 0 (no valid pixel in rows 0..k) has data cost 0; fO holds
            // byte offsets (mean - fbase) * 4 into the prior table
            const uint32_t fr = (uint32_t)mean_of(eA[t], eN[t], bcm[t]);
            const float d = po_at((fr << 8) + lane4b, bsb[t]);
            mO[t] = ((eN[t] == 0) ? 0.0f : d) + P.first[0];
            fO[t] = (eN[t] == 0) ? 0 : (int)(fr << 2) + bqo[t];
        } else {
            const int fi = mean_of(eA[t], eN[t], cmean);
            mO[t] = po_at(__umul24((uint32_t)fi, pstride4) + (uint32_t)kk * 4u, 0u) + P.first[0];
            fO[t] = fi;
        }
    }

    // The object prefix column at the current base, PO[fbase + 64c + lane][b],
    // is kept in registers and advanced by one row of the object cost table
    // per step (prefetched a step ahead); it never has to be gathered.  The
    // sky and ground prefixes and the ground-disparity bounds of the next
    // step are prefetched with it.  All go through buffer resources: unlike
    // flat loads they do not hold up the waits on this step's LDS traffic.
    float pcol[NCH], orow[NCH];
    int thi_n = 0, tlo_n = 0;
    float ps_n = 0.0f, pg_n = INF;
    const int nchunk = (nrow + 63) >> 6;             // 64-row chunks of disparity rows
    const auto odf = make_rsrc(in.O_df, (uint32_t)(in.D * in.D) * 4u);
    const auto fgh = make_rsrc(in.fg_hi, (uint32_t)H * 4u);
    const auto fgl = make_rsrc(in.fg_lo, (uint32_t)H * 4u);
    // per-lane byte offset of disparity row fbase + 64c + lane (2^30 past
    // the column's range); kept in registers for two chunks, recomputed per
    // step for four, where the registers are scarcer
    auto row_off = [&](int c) -> uint32_t {
        const int i = 64 * c + lane;
        return (i < nrow) ? (uint32_t)(fbase + i) * 4u : 0x40000000u;
    };
    uint32_t roff[NCH];
#pragma unroll
    for (int c = 0; c < NCH; ++c) roff[c] = row_off(c);
    // Short columns (S <= 8) read wave-uniform values of the 64 steps
    // j = 64 sj + lane of a slot once, a lane per step: the pixel q_{j+1}
    // the step prefetches and, with BLOCKS, the sky and ground prefixes at
    // j+1 and the bounds of the base row j+1 (top-down row H-2-j; without
    // BLOCKS these four are prefetched a step ahead).  A step takes its own
    // with readlane (scalar registers); with BLOCKS only the object gathers
    // and the object-cost row are vector memory instructions of a step.
    constexpr bool QB = (S <= 8);                    // the pixel a slot at a time
    constexpr bool BLK = BLOCKS && QB;               // and the other four
    // PIPE: one-wave columns of up to 8 slots gather a step's object
    // prefixes one step early.  The gathers of step j (stixels starting at
    // b = j+1) depend only on row j's prefix values, never on a cost, so
    // step j issues them for step j+1 right after folding its own, and a
    // whole step of work covers their latency.  The slot also holds the
    // prefix values of row j+1 of each of its steps.
    constexpr bool PIPE = (W == 1) && QB;
    struct Blk {
        int q = 0, thi = 0, tlo = 0;
        float ps = 0.0f, pg = 0.0f;
        float na = 0.0f;                // PA and PN2 (RT: as eN) at j+2 (PIPE)
        NT nn = 0;
    };
    const auto par = make_rsrc(in.PA, stride4);
    const auto pnr = make_rsrc(in.PN2, stride4);
    auto load_block = [&](int sj) {
        Blk k;
        const int j = 64 * sj + lane;
        k.q = (j + 1 < H) ? (int)in.q[j + 1] : -1;
        if constexpr (PIPE) {
            const int kk = min(j + 2, H);
            k.na = buf_load(par, kk);
            if constexpr (RT) {
                k.nn = (int)buf_load(pnr, kk) * 2;
            } else {
                k.nn = buf_load(pnr, kk);
            }
        }
        if constexpr (BLK) {
            k.ps = buf_load(psr, j + 1);              // past the table: 0, never used
            k.pg = buf_load(pgr, j + 1);
            k.thi = __builtin_bit_cast(int, buf_load(fgh, H - 2 - j));
            k.tlo = __builtin_bit_cast(int, buf_load(fgl, H - 2 - j));
        }
        return k;
    };
    auto load_next = [&](int v, int qv) {
        // for step v (qv = q_v): object costs of pixel q_v for every
        // disparity row, the sky and ground prefixes at v+1 (ground INF
        // above vtop) and the bounds of the base row v+1 (top-down row
        // H-2-v).  Straight-line code: every index either lies inside its
        // table or falls past the end of its buffer resource, which reads 0
        // (v <= H-1 gives top-down row >= -1; an invalid pixel or a
        // disparity row past the column's range gives index -1).
        // Byte offset of O[qv][fbase + i]: a wave-uniform part plus a
        // per-lane part; an invalid pixel or a disparity row past the
        // column's range adds 2^30, far past the end of the resource (in the
        // per-lane offset, which the bounds check always covers)
        const uint32_t qoff = (qv >= 0) ? (uint32_t)__umul24(qv, in.D) * 4u : 0x40000000u;
#pragma unroll
        for (int c = 0; c < NCH; ++c)
            orow[c] = buf_load_b(odf, ((NCH <= 2) ? roff[c] : row_off(c)) + qoff, 0u);
        if constexpr (BLK) return;
        // v + 1 <= H: inside the prefix tables, so the offset may be scalar
        ps_n = buf_load_b(psr, 0u, (uint32_t)(v + 1) * 4u);
        const float pg = buf_load_b(pgr, 0u, (uint32_t)(v + 1) * 4u);
        pg_n = (v <= vtop) ? pg : INF;
        thi_n = __builtin_bit_cast(int, buf_load(fgh, H - 2 - v));
        tlo_n = __builtin_bit_cast(int, buf_load(fgl, H - 2 - v));
    };
#pragma unroll
    for (int c = 0; c < NCH; ++c) pcol[c] = orow[c] = 0.0f;
    if (H > 1) load_next(0, __builtin_amdgcn_readfirstlane((int)in.q[0]));

    // PIPE: the object prefix gathers of step 0 (base b = 1; row 0's prefix
    // values are lane 0 of slot 0)
    float pkP[PIPE ? SW : 1];
    int fSP[PIPE ? SW : 1];
    if constexpr (PIPE) {
        const float nA0 = readlane_f(eA[0], 0);
        const NT nN0 = readlane_n(eN[0], 0);
#pragma unroll
        for (int t = 0; t < SW; ++t) {
            if constexpr (BAND) {
                const uint32_t fr = (uint32_t)mean_of(eA[t] - nA0, eN[t] - nN0, bcm[t]);
                pkP[t] = po_at((fr << 8) + lane4b, bsb[t]);
                fSP[t] = (int)(fr << 2) + bqo[t];
            } else {
                const uint32_t fi = (uint32_t)mean_of(eA[t] - nA0, eN[t] - nN0, cmean);
                pkP[t] = po_at(__umul24(fi, pstride4) + lane4, (uint32_t)(t * 256));
                fSP[t] = (int)fi;
            }
        }
    }

    // The ground and sky data terms of a stixel [b, k] are prefix
    // differences whose b-side does not depend on k, and their priors depend
    // on b alone: GR^k = PG[k+1] + min over b <= k of (prior_g(b) - PG[b]),
    // and the same for SK (Eq. 5).  All values are exact on the cost grid,
    // so the two minima are kept as running wave-uniform values RG and RS,
    // and a row's ground and sky costs are written once, when the row is
    // reached, instead of being folded per row and per step.
    float RG = P.first[1], RS = P.first[2];
    int bRG = 0, bRS = 0;               // cut positions of the minima (LINKS)

    // Push-form recurrence: step j finalises row j and folds the stixels
    // that start at b = j+1 into every row k > j.  Per step, the prior of an
    // object stixel with mean f (min over the three predecessor classes,
    // with the ordering / diving / gravity penalties) minus PO[f][b] is
    // tabulated once over the column's disparity rows in LDS; a candidate is
    // then that entry plus one gathered PO[f][k+1].  All slots' gathers are
    // issued before any candidate is folded.  Steps where no ground stixel
    // can end at or below b-1 (b > vtop+1) skip the ground terms.  Slots
    // below the current row are skipped by uniform branches.
    // tj = sj / W, the owning wave's local slot of row j: a compile-time
    // constant at every call, so that row j's registers are read by one
    // readlane each (a run-time slot would read every slot and select)
    auto step = [&](auto gr_tag, const int sj, const int jl, const int tj, const Blk& blk) {
        constexpr bool GR = decltype(gr_tag)::value;
        const int j = sj * 64 + jl, b = j + 1;
        // row j's object cost, mean and prefix values, read from its owning
        // lane; the slot is chosen by wave-uniform branches (an indexed
        // choice would put the slot registers in scratch memory)
        float Co = 0.0f, bA = 0.0f;
        NT bN = 0;
        int fp = 0;
        auto read_row = [&]() {
#pragma unroll
            for (int t = 0; t < SW; ++t) {
                if (t == tj) {
                    Co = readlane_f(mO[t], jl);
                    fp = readlane_i(fO[t], jl);
                    if constexpr (!PIPE) {
                        bA = readlane_f(eA[t], jl);
                        bN = readlane_n(eN[t], jl);
                    }
                }
            }
        };
        if constexpr (W == 1) {
            read_row();
        } else {
            float* bc = L.bc[j & 1];
            if (wave == sj % W) {
                read_row();
                if (lane == 0) {
                    bc[0] = Co;
                    bc[1] = __builtin_bit_cast(float, fp);
                    bc[2] = bA;
                    bc[3] = __builtin_bit_cast(float, bN);
                }
            }
            __syncthreads();
            Co = bc[0];
            fp = __builtin_bit_cast(int, bc[1]);
            bA = bc[2];
            bN = __builtin_bit_cast(NT, bc[3]);
        }
        // the b-side object prefix column moves to PO[.][j+1]
#pragma unroll
        for (int c = 0; c < NCH; ++c) pcol[c] += orow[c];

        // With two disparity chunks and up to eight slots, the gathers of
        // every open slot are issued first (they depend on row j's prefix
        // values only, not on its costs), so that their latency overlaps the
        // prior table; elsewhere the registers this holds across the table
        // build spill (measured slower), and each group is gathered and
        // folded after it.  Slots of a group that lie past the column's height
        // fold values into rows that are never read (their gathers stay
        // inside the column's table or read 0 past its end, and their table
        // index is masked): skipping them one by one would cost more than
        // the work.  Groups bound the registers a tall column holds.
        constexpr int G = (SW <= 8) ? SW : 4;
        constexpr bool EARLY = (NCH == 2) && (S <= 8) && !PIPE;
        float pk[SW];
        int fS[SW];
        auto gather = [&](int g0) {
#pragma unroll
            for (int t = g0; t < g0 + G && t < SW; ++t) {
                const int s = t * W + wave;
                if (s < sj) continue;
                if constexpr (BAND) {
                    const uint32_t fr = (uint32_t)mean_of(eA[t] - bA, eN[t] - bN, bcm[t]);
                    pk[t] = po_at((fr << 8) + lane4b, bsb[t]);
                    fS[t] = (int)(fr << 2) + bqo[t];
                } else {
                    const uint32_t fi = (uint32_t)mean_of(eA[t] - bA, eN[t] - bN, cmean);
                    pk[t] = po_at(__umul24(fi, pstride4) + lane4, (uint32_t)(s * 256));
                    fS[t] = (int)fi;
                }
            }
        };
        auto fold = [&](int g0) {
            float qv[SW];
#pragma unroll
            for (int t = g0; t < g0 + G && t < SW; ++t) {
                if (t * W + wave < sj) continue;
                if constexpr (BAND) {
                    // byte offset (mean - fbase) * 4 >= -4: the table's padding
                    qv[t] = *reinterpret_cast<const float*>(reinterpret_cast<const char*>(qtab) + fS[t]);
                } else {
                    // fi < 64 NCH except, possibly, in rows past H
                    qv[t] = qtab[(uint32_t)fS[t] & (64u * NCH - 1u)];
                }
            }
#pragma unroll
            for (int t = g0; t < g0 + G && t < SW; ++t) {
                const int s = t * W + wave;
                if (s < sj) continue;
                const bool act = (s > sj) || (lane > jl);          // rows k > j only
                float cO = qv[t] + pk[t];
                cO = act ? cO : INF;
                const bool better = cO < mO[t];
                mO[t] = better ? cO : mO[t];
                fO[t] = better ? fS[t] : fO[t];
                if constexpr (LINKS) bO[t] = better ? b : bO[t];
            }
        };
        auto group_open = [&](int g0) {
            return g0 * W < nslots && (g0 + G - 1) * W + wave >= sj;
        };
        if constexpr (EARLY) {
            // Only the previous step's object-cost row is still in flight
            // here (issued a step ago).  Waiting for it now, explicitly,
            // keeps the compiler from placing that wait after the gathers
            // below, where the in-order memory counter would make it wait
            // for the gathers too (vmcnt(0), expcnt and lgkmcnt untouched).
            __builtin_amdgcn_s_waitcnt(0x0F70);
            if (group_open(0)) gather(0);
        }

        // row j's ground and sky costs (ground is INF above vtop: bG is),
        // recorded for the backtracking
        const float bS = BLK ? readlane_f(blk.ps, jl) : ps_n;
        const float bG = BLK ? ((j <= vtop) ? readlane_f(blk.pg, jl) : INF) : pg_n;
        const float Cg = bG + RG, Cs = bS + RS;
        if (wave == 0 && lane == 0) {
            L.crow_g[j] = Cg;
            L.crow_s[j] = Cs;
            if constexpr (LINKS) {
                L.lk.b[1][j] = (int16_t)bRG;
                L.lk.b[2][j] = (int16_t)bRS;
            }
        }
        // bounds at base row b
        const int thi = BLK ? readlane_i(blk.thi, jl) : thi_n;
        const int tlo = BLK ? readlane_i(blk.tlo, jl) : tlo_n;
        // pixel q_{j+1}, base b+1 (b <= H-1); tall columns read the pixel
        // from LDS (registers held across their runtime loop spill)
        const int qb = QB ? readlane_i(blk.q, jl) : (int)in.q[b];   // pixel q_b
        load_next(b, qb);

        const float XS =
            vmin(vmin(Co + P.trans[0][2], Cg + P.trans[1][2]), Cs + P.trans[2][2]) - bS;
        if constexpr (LINKS) bRS = (XS < RS) ? b : bRS;
        RS = vmin(RS, XS);
        const float Xoo = Co + P.trans[0][0];
        const float Xoo_p = Xoo + P.c_ord;
        const int tord = (BAND ? (fp >> 2) : fp) + fbase + P.tau_ord;
        const float Xso = Cs + P.trans[2][0];
        float XG = INF, Xgo = INF, Xgo_d = INF, Xgo_g = INF;
        if constexpr (GR) {
            XG = (b <= vtop)
                ? vmin(vmin(Co + P.trans[0][1], Cg + P.trans[1][1]), Cs + P.trans[2][1]) - bG
                : INF;
            if constexpr (LINKS) bRG = (XG < RG) ? b : bRG;
            RG = vmin(RG, XG);
            Xgo = Cg + P.trans[1][0];
            Xgo_d = Xgo + P.c_dive;
            Xgo_g = Xgo + P.c_grav;
        }
        // RT: the reciprocals of the next step's candidates (row j+1's
        // count), read before the table is written, so that their LDS
        // latency passes under it instead of in front of each gather
        float rP[(PIPE && RT) ? SW : 1];
        if constexpr (PIPE && RT) {
            const NT nN = readlane_n(blk.nn, jl);
#pragma unroll
            for (int t = 0; t < SW; ++t) {
                if (t < sj) continue;
                rP[t] = *reinterpret_cast<const float*>(reinterpret_cast<const char*>(rtab) +
                                                        (eN[t] - nN));
            }
        }
        // this wave's copy of the table (LDS accesses of one wave complete
        // in order, so no barrier guards it)
#pragma unroll
        for (int c = 0; c < NCH; ++c) {
            // two chunks are both built (one block, so that the compares and
            // selects of the two interleave); an unused chunk is never read
            if (NCH > 2 && c >= nchunk) break;
            const int f = fbase + 64 * c + lane;
            const float v1 = (f > tord) ? Xoo_p : Xoo;
            float pr;
            if constexpr (GR) {
                float v2 = (f < tlo) ? Xgo_g : Xgo;
                v2 = (f > thi) ? Xgo_d : v2;
                pr = vmin(vmin(v1, v2), Xso);
            } else {
                pr = vmin(v1, Xso);
            }
            qtab[64 * c + lane] = pr - pcol[c];
        }

        if constexpr (PIPE) {
            // fold the gathers issued a step ago, then issue the next
            // step's (base b+1: row j+1's prefix values); a slot that closes
            // with this step still gathers once, into rows never folded
            const float nA = readlane_f(blk.na, jl);
            const NT nN = readlane_n(blk.nn, jl);
            float qv[SW];
#pragma unroll
            for (int t = 0; t < SW; ++t) {
                if (t < sj) continue;
                if constexpr (BAND) {
                    // byte offset (mean - fbase) * 4 >= -4: the table's padding
                    qv[t] = *reinterpret_cast<const float*>(reinterpret_cast<const char*>(qtab) + fSP[t]);
                } else {
                    qv[t] = qtab[(uint32_t)fSP[t] & (64u * NCH - 1u)];
                }
            }
#pragma unroll
            for (int t = 0; t < SW; ++t) {
                if (t < sj) continue;
                const bool act = (t > sj) || (lane > jl);          // rows k > j only
                float cO = qv[t] + pkP[t];
                cO = act ? cO : INF;
                const bool better = cO < mO[t];
                mO[t] = better ? cO : mO[t];
                fO[t] = better ? fSP[t] : fO[t];
                if constexpr (LINKS) bO[t] = better ? b : bO[t];
                if constexpr (BAND) {
                    uint32_t fr;
                    if constexpr (RT) {
                        fr = (uint32_t)cvt_i32_nan0(__builtin_fmaf(eA[t] - nA, rP[t], bcm[t]));
                    } else {
                        fr = (uint32_t)mean_of(eA[t] - nA, eN[t] - nN, bcm[t]);
                    }
                    pkP[t] = po_at((fr << 8) + lane4b, bsb[t]);
                    fSP[t] = (int)(fr << 2) + bqo[t];
                } else {
                    const uint32_t fi = (uint32_t)mean_of(eA[t] - nA, eN[t] - nN, cmean);
                    pkP[t] = po_at(__umul24(fi, pstride4) + lane4, (uint32_t)(t * 256));
                    fSP[t] = (int)fi;
                }
            }
            if constexpr (BAND) {
                // stixels [b, k] without a valid pixel: pixel b is invalid,
                // so PN2 at b+1 (nN) equals PN2 at b
                if (qb < 0) {
                    const float v1 = (0 > tord) ? Xoo_p : Xoo;
                    float pr0;
                    if constexpr (GR) {
                        float v2 = (0 < tlo) ? Xgo_g : Xgo;
                        v2 = (0 > thi) ? Xgo_d : v2;
                        pr0 = vmin(vmin(v1, v2), Xso);
                    } else {
                        pr0 = vmin(v1, Xso);
                    }
#pragma unroll
                    for (int t = 0; t < SW; ++t) {
                        if (t < sj) continue;
                        const bool act = ((t > sj) || (lane > jl)) && (eN[t] == nN);
                        const bool better = act && (pr0 < mO[t]);
                        mO[t] = better ? pr0 : mO[t];
                        fO[t] = better ? 0 : fO[t];
                    }
                }
            }
        } else if constexpr (EARLY) {
            if (group_open(0)) fold(0);
            if constexpr (BAND) {
                // stixels [b, k] without a valid pixel (pixel b invalid, n = 0)
                // have mean 0, data cost 0 and cost the prior at mean 0 (fbase
                // is 0 whenever the column holds an invalid pixel); their
                // gathers read the +inf row, so they are folded here
                if (qb < 0) {
                    const float v1 = (0 > tord) ? Xoo_p : Xoo;
                    float pr0;
                    if constexpr (GR) {
                        float v2 = (0 < tlo) ? Xgo_g : Xgo;
                        v2 = (0 > thi) ? Xgo_d : v2;
                        pr0 = vmin(vmin(v1, v2), Xso);
                    } else {
                        pr0 = vmin(v1, Xso);
                    }
#pragma unroll
                    for (int t = 0; t < SW; ++t) {
                        const int s = t * W + wave;
                        if (s < sj) continue;
                        const bool act = ((s > sj) || (lane > jl)) && (eN[t] == bN);
                        const bool better = act && (pr0 < mO[t]);
                        mO[t] = better ? pr0 : mO[t];
                        fO[t] = better ? 0 : fO[t];
                    }
                }
            }
        } else {
#pragma unroll
            for (int g0 = 0; g0 < SW; g0 += G) {
                if (g0 * W >= nslots) break;
                if (!group_open(g0)) continue;
                gather(g0);
                fold(g0);
            }
            if constexpr (BAND) {
                // stixels [b, k] without a valid pixel (pixel b invalid, n = 0)
                // have mean 0, data cost 0 and cost the prior at mean 0 (fbase
                // is 0 whenever the column holds an invalid pixel); their
                // gathers read the +inf row, so they are folded here
                if (qb < 0) {
                    const float v1 = (0 > tord) ? Xoo_p : Xoo;
                    float pr0;
                    if constexpr (GR) {
                        float v2 = (0 < tlo) ? Xgo_g : Xgo;
                        v2 = (0 > thi) ? Xgo_d : v2;
                        pr0 = vmin(vmin(v1, v2), Xso);
                    } else {
                        pr0 = vmin(v1, Xso);
                    }
#pragma unroll
                    for (int t = 0; t < SW; ++t) {
                        const int s = t * W + wave;
                        if (s < sj) continue;
                        const bool act = ((s > sj) || (lane > jl)) && (eN[t] == bN);
                        const bool better = act && (pr0 < mO[t]);
                        mO[t] = better ? pr0 : mO[t];
                        fO[t] = better ? 0 : fO[t];
                    }
                }
            }
        }
    };

    if constexpr (S <= 8) {
        // unrolled over the slot of row j, so that every slot test above is
        // decided at compile time (for W = 1) and the slots' gathers share
        // one block
#pragma unroll
        for (int sj = 0; sj < S; ++sj) {
            const int jend = min(64, H - 1 - sj * 64);
            if (jend <= 0) break;
            const Blk blk = load_block(sj);
            // the slot's values are in registers before its steps start;
            // otherwise the compiler's wait counts inside the step, which
            // cannot tell the loop's iterations apart, would also wait for
            // most of the step's own gathers before reading them
            __builtin_amdgcn_s_waitcnt(0);
            // steps whose base b = sj*64+jl+1 can still follow a ground stixel
            const int jgr = min(jend, max(0, vtop + 1 - sj * 64));
            for (int jl = 0; jl < jgr; ++jl) step(std::true_type{}, sj, jl, sj / W, blk);
            for (int jl = jgr; jl < jend; ++jl) step(std::false_type{}, sj, jl, sj / W, blk);
        }
    } else if constexpr (SW <= 8) {
        // tall columns shared by several waves: one copy of the step per
        // local slot of row j's owner (at most 8, as for short columns),
        // the owning wave a run-time loop
        const Blk none;
        static_for<0, SW>([&](auto tc) {
            constexpr int T = decltype(tc)::value;
            for (int wj = 0; wj < W; ++wj) {
                const int sj = T * W + wj;
                const int jend = min(64, H - 1 - sj * 64);
                if (jend <= 0) break;
                const int jgr = min(jend, max(0, vtop + 1 - sj * 64));
                for (int jl = 0; jl < jgr; ++jl) step(std::true_type{}, sj, jl, T, none);
                for (int jl = jgr; jl < jend; ++jl) step(std::false_type{}, sj, jl, T, none);
            }
        });
    } else {
        // tall one-wave columns: one runtime loop keeps the code (and the
        // registers live across it) to a single copy of the step
        const Blk none;
        for (int j = 0; j < H - 1; ++j) {
            if (j + 1 <= vtop + 1) step(std::true_type{}, j >> 6, j & 63, (j >> 6) / W, none);
            else step(std::false_type{}, j >> 6, j & 63, (j >> 6) / W, none);
        }
    }

    // the top row's ground and sky costs, and every row's object cost and
    // mean, into LDS for the backtracking.  Callers may keep the column's
    // pixels (in.q) in the crow_o array until here: with several waves, no
    // wave overwrites it before all have left the recurrence
    if constexpr (W > 1) __syncthreads();
    if (wave == 0 && lane == 0) {
        L.crow_g[H - 1] = ((H - 1 <= vtop) ? buf_load(pgr, H) : INF) + RG;
        L.crow_s[H - 1] = buf_load(psr, H) + RS;
        if constexpr (LINKS) {
            L.lk.b[1][H - 1] = (int16_t)bRG;
            L.lk.b[2][H - 1] = (int16_t)bRS;
        }
    }
#pragma unroll
    for (int t = 0; t < SW; ++t) {
        const int s = t * W + wave;
        if (s < S) {
            L.crow_o[s * 64 + lane] = mO[t];
            L.crow_f[s * 64 + lane] = (uint8_t)(BAND ? (fO[t] >> 2) : fO[t]);
            if constexpr (LINKS) L.lk.b[0][s * 64 + lane] = (int16_t)bO[t];
        }
    }
    __syncthreads();
    if (wave != 0) return;
#ifdef STX_PHASE_TIMING
    if (lane == 0 && out.t_rec_end) *out.t_rec_end = __builtin_amdgcn_s_memtime();
#endif

    if constexpr (LINKS) {
        backtrack_links<S>(H, vtop, P, in, out, L);
    } else {
        backtrack_column<S, ColumnLds<S, W, 64 * NCH, LINKS>, BAND>(H, vtop, P, in, out, L);
    }
}


// Two columns of one frame per wave64 (same height, same camera model): the
// lanes of half X = lane / 32 take column X, and lane l of that half owns
// rows k = 32 s + l for 32-row slots s < 2 S.  Every per-step operation of
// solve_column (the row broadcast, the prior table, the running minima, the
// prefetch) then serves two columns at once.  The two columns' tables lie
// one column stride apart (in1.X = in0.X + the stride for every table, PO
// after eight (h+1) arrays: PG, PS, PA, PN and the four row-cost arrays).
// has1: the second column exists (a frame with an odd column count leaves
// the last pair's second half idle; its results are not written).
// qs2: the two columns' reduced pixels in LDS, [2][64 S].
template <int S, int NCH>
__device__ __forceinline__ void solve_pair(const int H, const int vtop, const Prior P, const ColumnIn& in0,
                           const ColumnIn& in1, const ColumnOut& out0, const ColumnOut& out1,
                           const bool has1, const int16_t* qs2, float* qtab2,
                           ColumnLds<S, 1>& L) {
    constexpr int S2 = 2 * S;                        // 32-row slots
    constexpr int NC = 2 * NCH;                      // 32-entry disparity chunks
    const int lane = threadIdx.x & 63;
    const int X = lane >> 5, l = lane & 31;
    const int stride = H + 1;
    const uint32_t stride4 = (uint32_t)stride * 4u;
    const uint32_t colstride4 = (uint32_t)(in1.PG - in0.PG) * 4u;
    const uint32_t cb = X ? colstride4 : 0u;         // this half's column base (bytes)
    const auto tab = make_rsrc(in0.PG, 2u * colstride4);
    const uint32_t oPG = cb, oPS = cb + stride4, oPA = cb + 2u * stride4, oPN = cb + 3u * stride4;
    const uint32_t oRO = cb + 4u * stride4, oRG = cb + 5u * stride4, oRS = cb + 6u * stride4,
                   oRF = cb + 7u * stride4, oPO = cb + 8u * stride4;
    const int fbase = X ? in1.fbase : in0.fbase;
    const int nrow = (X ? in1.fmax : in0.fmax) - fbase + 1;
    // 32-entry chunks of disparity rows that either column needs
    const int nchunk = max(__builtin_amdgcn_readlane((nrow + 31) >> 5, 0),
                           __builtin_amdgcn_readlane((nrow + 31) >> 5, 32));
    const float eps = P.mean_eps;
    const float cmean = eps - (float)fbase;
    const float INF = inf_f();
    const uint32_t lanek4 = oPO + (uint32_t)(l + 1) * 4u;   // PO row offset of k+1 within slot 0
    float* const qtab = qtab2 + X * 256;

    float eA[S2], eN[S2], mO[S2];
    int fO[S2];
    const int nslots = (H + 31) >> 5;

#pragma unroll
    for (int t = 0; t < S2; ++t) {
        if (t >= nslots) {
            mO[t] = INF;
            eA[t] = eN[t] = 0.0f;
            fO[t] = 0;
            continue;
        }
        const int k = t * 32 + l;
        const int kk = min(k + 1, H);
        eA[t] = buf_load_b(tab, oPA + (uint32_t)kk * 4u, 0u);
        eN[t] = buf_load_b(tab, oPN + (uint32_t)kk * 4u, 0u);
        const int fi = mean_index(eA[t], eN[t], cmean);
        mO[t] = buf_load_b(tab, oPO + __umul24((uint32_t)fi, stride4) + (uint32_t)kk * 4u, 0u) +
                P.first[0];
        fO[t] = fi;
    }

    float pcol[NC], orow[NC];
    uint32_t roff[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        const int i = 32 * c + l;
        roff[c] = (i < nrow) ? (uint32_t)(fbase + i) * 4u : 0x40000000u;
        pcol[c] = orow[c] = 0.0f;
    }
    int thi_n = 0, tlo_n = 0;
    float ps_n = 0.0f, pg_n = INF;
    const auto odf = make_rsrc(in0.O_df, (uint32_t)(in0.D * in0.D) * 4u);
    const auto fgh = make_rsrc(in0.fg_hi, (uint32_t)H * 4u);
    const auto fgl = make_rsrc(in0.fg_lo, (uint32_t)H * 4u);
    auto load_next = [&](int v) {
        const int qv = qs2[X * 64 * S + v];
        const uint32_t qoff = (qv >= 0) ? (uint32_t)(qv * in0.D) * 4u : 0x40000000u;
#pragma unroll
        for (int c = 0; c < NC; ++c) orow[c] = buf_load_b(odf, roff[c] + qoff, 0u);
        ps_n = buf_load_b(tab, oPS + (uint32_t)(v + 1) * 4u, 0u);
        const float pg = buf_load_b(tab, oPG + (uint32_t)(v + 1) * 4u, 0u);
        pg_n = (v <= vtop) ? pg : INF;
        thi_n = __builtin_bit_cast(int, buf_load(fgh, H - 2 - v));
        tlo_n = __builtin_bit_cast(int, buf_load(fgl, H - 2 - v));
    };
    if (H > 1) load_next(0);

    float RG = P.first[1], RS = P.first[2];   // running minima (separable ground and sky terms)

    // one step: row j = 32 sj + jl of both columns is final; fold the stixels
    // starting at b = j + 1 into the rows k > j
    auto step = [&](auto gr_tag, const int sj, const int jl) {
        constexpr bool GR = decltype(gr_tag)::value;
        const int j = sj * 32 + jl, b = j + 1;
        float Co = 0.0f, bA = 0.0f, bN = 0.0f;
        int fp = 0;
#pragma unroll
        for (int t = 0; t < S2; ++t) {
            if (t == sj) {
                const float c0 = readlane_f(mO[t], jl), c1 = readlane_f(mO[t], jl + 32);
                const int f0 = readlane_i(fO[t], jl), f1 = readlane_i(fO[t], jl + 32);
                const float a0 = readlane_f(eA[t], jl), a1 = readlane_f(eA[t], jl + 32);
                const float n0 = readlane_f(eN[t], jl), n1 = readlane_f(eN[t], jl + 32);
                Co = X ? c1 : c0;
                fp = X ? f1 : f0;
                bA = X ? a1 : a0;
                bN = X ? n1 : n0;
            }
        }
        const float bS = ps_n, bG = pg_n;
        const float Cg = bG + RG, Cs = bS + RS;
        if (l == 0) {   // row j's ground and sky costs, for the backtracking
            buf_store_b(tab, Cg, oRG + (uint32_t)j * 4u, 0u);
            buf_store_b(tab, Cs, oRS + (uint32_t)j * 4u, 0u);
        }
#pragma unroll
        for (int c = 0; c < NC; ++c) pcol[c] += orow[c];
        const int thi = thi_n, tlo = tlo_n;
        load_next(b);

        const float XS =
            vmin(vmin(Co + P.trans[0][2], Cg + P.trans[1][2]), Cs + P.trans[2][2]) - bS;
        RS = vmin(RS, XS);
        const float Xoo = Co + P.trans[0][0];
        const float Xoo_p = Xoo + P.c_ord;
        const int tord = fp + fbase + P.tau_ord;
        const float Xso = Cs + P.trans[2][0];
        float Xgo = INF, Xgo_d = INF, Xgo_g = INF;
        if constexpr (GR) {
            const float XG = (b <= vtop)
                ? vmin(vmin(Co + P.trans[0][1], Cg + P.trans[1][1]), Cs + P.trans[2][1]) - bG
                : INF;
            RG = vmin(RG, XG);
            Xgo = Cg + P.trans[1][0];
            Xgo_d = Xgo + P.c_dive;
            Xgo_g = Xgo + P.c_grav;
        }
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            if (c >= nchunk) break;
            const int f = fbase + 32 * c + l;
            const float v1 = (f > tord) ? Xoo_p : Xoo;
            float pr;
            if constexpr (GR) {
                float v2 = (f < tlo) ? Xgo_g : Xgo;
                v2 = (f > thi) ? Xgo_d : v2;
                pr = vmin(vmin(v1, v2), Xso);
            } else {
                pr = vmin(v1, Xso);
            }
            qtab[32 * c + l] = pr - pcol[c];
        }

        float pk[S2], qv[S2];
        int fS[S2];
        constexpr int G = (S2 <= 8) ? S2 : 8;
#pragma unroll
        for (int g0 = 0; g0 < S2; g0 += G) {
            if (g0 >= nslots) break;
            if (g0 + G <= sj) continue;
#pragma unroll
            for (int t = g0; t < g0 + G && t < S2; ++t) {
                if (t < sj) continue;
                const uint32_t fi = (uint32_t)mean_index(eA[t] - bA, eN[t] - bN, cmean);
                pk[t] = buf_load_b(tab, __umul24(fi, stride4) + lanek4, (uint32_t)(t * 128));
                qv[t] = qtab[fi & 255u];
                fS[t] = (int)fi;
            }
#pragma unroll
            for (int t = g0; t < g0 + G && t < S2; ++t) {
                if (t < sj) continue;
                const bool act = (t > sj) || (l > jl);
                float cO = qv[t] + pk[t];
                cO = act ? cO : INF;
                const bool better = cO < mO[t];
                mO[t] = better ? cO : mO[t];
                fO[t] = better ? fS[t] : fO[t];
            }
        }
    };

    // unrolled over the 32-row slot of row j, so that every slot test is
    // decided at compile time
#pragma unroll
    for (int sj = 0; sj < S2; ++sj) {
        const int jend = min(32, H - 1 - sj * 32);
        const int jgr = min(jend, max(0, vtop + 1 - sj * 32));
        for (int jl = 0; jl < jgr; ++jl) step(std::true_type{}, sj, jl);
        for (int jl = jgr; jl < jend; ++jl) step(std::false_type{}, sj, jl);
    }

    // the top rows' ground and sky costs, and every row's object cost and
    // best mean, into the row-cost arrays
    if (l == 0) {
        const float pg = buf_load_b(tab, oPG + (uint32_t)H * 4u, 0u);
        buf_store_b(tab, ((H - 1 <= vtop) ? pg : INF) + RG, oRG + (uint32_t)(H - 1) * 4u, 0u);
        buf_store_b(tab, buf_load_b(tab, oPS + (uint32_t)H * 4u, 0u) + RS,
                    oRS + (uint32_t)(H - 1) * 4u, 0u);
    }
#pragma unroll
    for (int t = 0; t < S2; ++t) {
        const int k = t * 32 + l;
        if (t < nslots && k < H) {
            buf_store_b(tab, mO[t], oRO + (uint32_t)k * 4u, 0u);
            buf_store_b(tab, __builtin_bit_cast(float, fO[t]), oRF + (uint32_t)k * 4u, 0u);
        }
    }

    // backtracking, one column at a time over the whole wave, from LDS copies
    // of the row costs (the barrier orders the stores above before the loads
    // below, which other lanes make)
    __syncthreads();
    for (int x = 0; x < 2; ++x) {
        if (x == 1 && !has1) break;
        const ColumnIn& in = x ? in1 : in0;
        const float* rc = in.rowc;
        for (int k = lane; k < H; k += 64) {
            L.crow_o[k] = rc[k];
            L.crow_g[k] = rc[stride + k];
            L.crow_s[k] = rc[2 * stride + k];
            L.crow_f[k] = (uint8_t)__builtin_bit_cast(int, rc[3 * stride + k]);
        }
        __syncthreads();
        backtrack_column<S>(H, vtop, P, in, x ? out1 : out0, L);
        __syncthreads();
    }
}

}  // namespace stx
