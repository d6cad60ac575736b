// Coupling kernels of the mixed FP32 precision (Sect. 2.6, M2L); the device
// code is shared with the other precisions.
#include "m2l_device.hpp"

namespace fdm {

namespace {

FDM_M2L_KERNEL(k_m2l_f32, F32SharedW, item_f32k, true)
FDM_M2L_LAUNCHERS(k_m2l_f32, launch_items_f32, resident_f32, false)

}  // namespace

}  // namespace fdm
