// kernel_table.h -- host pointers of the instantiated recurrence kernels.
//
// The kernel templates (batch_kernel.h, dp_kernel.h) are instantiated per
// slot count in the inst_s*.hip units, so that the many variants compile in
// parallel; launchers look a variant up here and start it with
// hipLaunchKernel.  Every lookup returns nullptr for a variant that does not
// exist.
#pragma once

namespace stx {

// Slot counts that have kernels (64-row slots per lane: kernel_slots()).
#define STX_FOR_EACH_SLOTS(X) X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(10) X(12) X(14) X(16)

#define STX_DECLARE_SLOTS(n)                                                   \
    const void* batch_kernel_ptr_s##n(int nch, int waves);                     \
    const void* batch_links_kernel_ptr_s##n(int nch);                          \
    const void* batch_pair_kernel_ptr_s##n(int nch);                           \
    const void* dp_kernel_ptr_s##n(int nch, int waves, bool pol);
STX_FOR_EACH_SLOTS(STX_DECLARE_SLOTS)
#undef STX_DECLARE_SLOTS

// persistent batched kernel <slots, disparity chunks, waves per column>
const void* batch_kernel_ptr(int slots, int nch, int waves);
// persistent batched kernel with stored links, one wave per column
// <slots, disparity chunks> (costs off the grid)
const void* batch_links_kernel_ptr(int slots, int nch);
// two columns per wave <slots, disparity chunks>
const void* batch_pair_kernel_ptr(int slots, int nch);
// staged per-frame recurrence <slots, disparity chunks, waves, LDS table copy>
const void* dp_kernel_ptr(int slots, int nch, int waves, bool pol);

}  // namespace stx
