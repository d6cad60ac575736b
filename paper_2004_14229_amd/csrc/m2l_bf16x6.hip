// Coupling kernels of the six-product BF16 split precision (Sect. 2.6, M2L);
// the device code is shared with the other precisions.
#include "m2l_device.hpp"

namespace fdm {

namespace {

FDM_M2L_KERNEL(k_m2l_bf16x6, BF16x6Shared, item_bf16x6k, true)
FDM_M2L_LAUNCHERS(k_m2l_bf16x6, launch_items_bf16x6, resident_bf16x6, false)

}  // namespace

}  // namespace fdm
