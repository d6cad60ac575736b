// Coupling kernels of the BF16 hi/lo split precision (Sect. 2.6, M2L); the device
// code is shared with the other precisions.
#include "m2l_device.hpp"

namespace fdm {

namespace {

FDM_M2L_KERNEL(k_m2l_bf16x3, BF16Shared, item_bf16k, true)
FDM_M2L_LAUNCHERS(k_m2l_bf16x3, launch_items_bf16, resident_bf16, false)

}  // namespace

}  // namespace fdm
