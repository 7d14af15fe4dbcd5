// kernel_table.hip -- dispatch of kernel lookups to the per-slot-count units.
#include "kernel_table.h"

namespace stx {

const void* batch_kernel_ptr(int slots, int nch, int waves) {
    switch (slots) {
#define STX_CASE(n) case n: return batch_kernel_ptr_s##n(nch, waves);
        STX_FOR_EACH_SLOTS(STX_CASE)
#undef STX_CASE
        default: return nullptr;
    }
}

const void* batch_links_kernel_ptr(int slots, int nch) {
    switch (slots) {
#define STX_CASE(n) case n: return batch_links_kernel_ptr_s##n(nch);
        STX_FOR_EACH_SLOTS(STX_CASE)
#undef STX_CASE
        default: return nullptr;
    }
}

const void* batch_pair_kernel_ptr(int slots, int nch) {
    switch (slots) {
#define STX_CASE(n) case n: return batch_pair_kernel_ptr_s##n(nch);
        STX_FOR_EACH_SLOTS(STX_CASE)
#undef STX_CASE
        default: return nullptr;
    }
}

const void* dp_kernel_ptr(int slots, int nch, int waves, bool pol) {
    switch (slots) {
#define STX_CASE(n) case n: return dp_kernel_ptr_s##n(nch, waves, pol);
        STX_FOR_EACH_SLOTS(STX_CASE)
#undef STX_CASE
        default: return nullptr;
    }
}

}  // namespace stx
