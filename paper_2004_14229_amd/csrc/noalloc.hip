// Allocation-free matvec: fdm_plan_matvec for plans with a streamed coupling
// bank, with the bank generated into a static workspace of the library
// instead of a workspace the plan allocates.
//
// The workspace is a file-scope device array, one copy per GPU, held until
// the process ends.  Host code never passes the array's name to a kernel
// (on the host it is only a stand-in for the symbol): its device address is
// looked up once per device with hipGetSymbolAddress, with that device
// current, when a plan on that device builds its launch schedule (plan
// set-up), and kept per device.  Every allocation-free matvec on a device
// shares that device's copy, so such calls on one device must not overlap.
// Nothing in the workspace needs to start at zero: each coupling launch
// writes every entry of the matrices it generates before its items read
// them.
#include <mutex>

#include "plan.hpp"
#include "capi.hpp"

namespace fdm {

namespace {

constexpr int64_t kStaticWorkspaceBytes = int64_t(64) << 20;  // 64 MiB per GPU
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kStaticWorkspaceBytes];

std::mutex g_scratch_mutex;
void* g_scratch_ptr[kMaxDevices] = {};

}  // namespace

int64_t static_workspace_bytes() { return kStaticWorkspaceBytes; }

void* static_workspace() {
  int dev = 0;
  FDM_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) fail(FDM_ERR_UNSUPPORTED, "device index out of range");
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    FDM_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    if (!ptr) fail(FDM_ERR_HIP, "hipGetSymbolAddress returned no address for the workspace");
    g_scratch_ptr[dev] = ptr;
  }
  return g_scratch_ptr[dev];
}

}  // namespace fdm

using namespace fdm;

extern "C" int fdm_plan_matvec_noalloc(fdm_plan* plan, const void* v, void* y, int c64,
                                       void* stream) {
  return guarded([&] {
    if (!plan) fail(FDM_ERR_INVALID_ARG, "plan is NULL");
    Plan& P = plan->p;
    if (c64 != 0 && c64 != 1) fail(FDM_ERR_INVALID_ARG, "c64 must be 0 or 1");
    if (P.bank_budget <= 0)
      fail(FDM_ERR_INVALID_ARG, "the plan's coupling bank is resident: use fdm_plan_matvec");
    const int64_t need = plan_workspace_bytes(P);
    if (need > static_workspace_bytes())
      fail(FDM_ERR_INVALID_ARG,
           "the plan's bank workspace (" + std::to_string(need) +
               " bytes) exceeds the static workspace (" +
               std::to_string(static_workspace_bytes()) + " bytes): build it with a smaller "
               "bank_budget_bytes");
    if (P.nS) check_device_ptr(v, "v");
    if (P.nT) check_device_ptr(y, "y");
    const int64_t w = c64 ? 8 : 16;
    if (P.nS && P.nT) {
      const char* a = static_cast<const char*>(v);
      const char* b = static_cast<const char*>(y);
      if (a < b + w * P.nT && b < a + w * P.nS) fail(FDM_ERR_INVALID_ARG, "v and y overlap");
    }
    if (P.nT && P.nS && (!P.sched_ready || (need > 0 && !P.static_ready)))
      fail(FDM_ERR_STATE, "the plan is not prepared: call fdm_plan_prepare first");
    plan_matvec(P, v, y, c64 != 0, static_cast<hipStream_t>(stream), need > 0);
  });
}
