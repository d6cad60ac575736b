// Coupling kernels of the plain FP64 precision (Sect. 2.6, M2L); the device
// code is shared with the other precisions.
#include "m2l_device.hpp"

namespace fdm {

namespace {

FDM_M2L_KERNEL(k_m2l_f64, F64Shared, item_f64, false)
FDM_M2L_LAUNCHERS(k_m2l_f64, launch_items_f64, resident_f64, true)

}  // namespace

}  // namespace fdm
