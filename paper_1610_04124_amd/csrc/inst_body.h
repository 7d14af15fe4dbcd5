// inst_body.h -- instantiates the recurrence kernels of one slot count
// (STX_SLOTS, defined by the including inst_s*.hip unit) and defines that
// slot count's lookups of kernel_table.h.
#pragma once

#include "batch_kernel.h"
#include "dp_kernel.h"
#include "kernel_table.h"

#ifndef STX_SLOTS
#error "define STX_SLOTS before including inst_body.h"
#endif

#define STX_CAT2(a, b) a##b
#define STX_CAT(a, b) STX_CAT2(a, b)

namespace stx {
namespace {

// Inside a template, the branch `if constexpr` discards is not instantiated:
// each unit instantiates the variants of its own slot count only.
template <int N, int C, int W>
const void* pick_batch(int nch, int waves) {
    if constexpr (N == STX_SLOTS) {
        if (nch == C && waves == W) return reinterpret_cast<const void*>(&persist::batch_kernel<N, C, W>);
    }
    return nullptr;
}

template <int N, int C>
const void* pick_links(int nch) {
    if constexpr (N == STX_SLOTS) {
        if (nch == C) return reinterpret_cast<const void*>(&persist::batch_kernel<N, C, 1, true>);
    }
    return nullptr;
}

template <int N, int C>
const void* pick_pair(int nch) {
    if constexpr (N == STX_SLOTS) {
        if (nch == C) return reinterpret_cast<const void*>(&persist::batch_pair_kernel<N, C>);
    }
    return nullptr;
}

template <int N, int C, int W>
const void* pick_dp(int nch, int waves, bool pol) {
    if constexpr (N == STX_SLOTS) {
        if (nch == C && waves == W) {
            // the LDS table copy exists for one wave per column, d_range <= 128
            // and up to 8 slots only
            if constexpr (N <= 8 && C == 2 && W == 1) {
                if (pol) return reinterpret_cast<const void*>(&dp_kernel<N, C, W, true>);
            }
            return pol ? nullptr : reinterpret_cast<const void*>(&dp_kernel<N, C, W, false>);
        }
    }
    return nullptr;
}

}  // namespace

const void* STX_CAT(batch_kernel_ptr_s, STX_SLOTS)(int nch, int waves) {
#define STX_CASE(n, c, w) \
    if (const void* p = pick_batch<n, c, w>(nch, waves)) return p;
    STX_FOR_EACH_VARIANT(STX_CASE)
#undef STX_CASE
    return nullptr;
}

const void* STX_CAT(batch_links_kernel_ptr_s, STX_SLOTS)(int nch) {
#define STX_CASE(n, c) \
    if (const void* p = pick_links<n, c>(nch)) return p;
    STX_FOR_EACH_LINKS_VARIANT(STX_CASE)
#undef STX_CASE
    return nullptr;
}

const void* STX_CAT(batch_pair_kernel_ptr_s, STX_SLOTS)(int nch) {
#define STX_CASE(n, c) \
    if (const void* p = pick_pair<n, c>(nch)) return p;
    STX_FOR_EACH_PAIR_VARIANT(STX_CASE)
#undef STX_CASE
    return nullptr;
}

const void* STX_CAT(dp_kernel_ptr_s, STX_SLOTS)(int nch, int waves, bool pol) {
#define STX_CASE(n, c, w) \
    if (const void* p = pick_dp<n, c, w>(nch, waves, pol)) return p;
    STX_FOR_EACH_VARIANT(STX_CASE)
#undef STX_CASE
    return nullptr;
}

}  // namespace stx
