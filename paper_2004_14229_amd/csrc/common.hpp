// Shared host/device utilities of the fdm library (gfx950 only).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
#include <stdexcept>
#include <string>
#include <utility>
#include <vector>

#include "../../include/fdm.h"

namespace fdm {

// Error carrying an fdm_status; converted to a return code at the C ABI.
struct Error : std::runtime_error {
  int status;
  Error(int s, const std::string& msg) : std::runtime_error(msg), status(s) {}
};

[[noreturn]] inline void fail(int status, const std::string& msg) {
  throw Error(status, msg);
}

inline void hip_check(hipError_t e, const char* what) {
  if (e == hipSuccess) return;
  if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation)
    fail(FDM_ERR_OUT_OF_MEMORY, std::string(what) + ": out of device memory");
  fail(FDM_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}
#define FDM_HIP(call) ::fdm::hip_check((call), #call)
#define FDM_LAUNCH(what) ::fdm::hip_check(hipGetLastError(), what)

// Owning device buffer; counts its bytes into a per-plan tally.
template <class T>
class DevBuf {
 public:
  DevBuf() = default;
  explicit DevBuf(size_t n, int64_t* tally = nullptr) { alloc(n, tally); }
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  DevBuf(DevBuf&& o) noexcept { swap(o); }
  DevBuf& operator=(DevBuf&& o) noexcept {
    if (this != &o) { release(); swap(o); }
    return *this;
  }
  ~DevBuf() { release(); }

  void alloc(size_t n, int64_t* tally = nullptr) {
    release();
    if (n == 0) return;
    void* p = nullptr;
    FDM_HIP(hipMalloc(&p, n * sizeof(T)));
    ptr_ = static_cast<T*>(p);
    n_ = n;
    tally_ = tally;
    if (tally_) *tally_ += static_cast<int64_t>(n * sizeof(T));
  }
  void release() {
    if (ptr_) {
      (void)hipFree(ptr_);
      if (tally_) *tally_ -= static_cast<int64_t>(n_ * sizeof(T));
    }
    ptr_ = nullptr;
    n_ = 0;
    tally_ = nullptr;
  }
  T* get() const { return ptr_; }
  size_t size() const { return n_; }
  size_t bytes() const { return n_ * sizeof(T); }

 private:
  void swap(DevBuf& o) {
    std::swap(ptr_, o.ptr_);
    std::swap(n_, o.n_);
    std::swap(tally_, o.tally_);
  }
  T* ptr_ = nullptr;
  size_t n_ = 0;
  int64_t* tally_ = nullptr;
};

template <class T>
void to_device(DevBuf<T>& d, const std::vector<T>& h, hipStream_t s,
               int64_t* tally) {
  d.alloc(h.size(), tally);
  if (!h.empty())
    FDM_HIP(hipMemcpyAsync(d.get(), h.data(), h.size() * sizeof(T),
                           hipMemcpyHostToDevice, s));
}

template <class T>
std::vector<T> to_host(const T* d, size_t n, hipStream_t s) {
  std::vector<T> h(n);
  if (n) {
    FDM_HIP(hipMemcpyAsync(h.data(), d, n * sizeof(T), hipMemcpyDeviceToHost, s));
    FDM_HIP(hipStreamSynchronize(s));
  }
  return h;
}

inline unsigned grid_for(int64_t n, int block) {
  int64_t g = (n + block - 1) / block;
  if (g < 1) g = 1;
  if (g > 1 << 20) g = 1 << 20;  // grid-stride loops cover the rest
  return static_cast<unsigned>(g);
}

// Morton code of 3 integer coordinates with `level` bits each; the x bit is
// the most significant of every octal digit (octant = 4*bx + 2*by + bz).
__host__ __device__ inline uint32_t morton3(uint32_t ix, uint32_t iy,
                                            uint32_t iz, int level) {
  uint32_t key = 0;
  for (int b = level - 1; b >= 0; --b)
    key = (key << 3) | (((ix >> b) & 1u) << 2) | (((iy >> b) & 1u) << 1) |
          ((iz >> b) & 1u);
  return key;
}

__host__ __device__ inline void demorton3(uint32_t key, int level, int& ix,
                                          int& iy, int& iz) {
  ix = iy = iz = 0;
  for (int b = 0; b < level; ++b) {
    uint32_t oct = (key >> (3 * b)) & 7u;
    ix |= int((oct >> 2) & 1u) << b;
    iy |= int((oct >> 1) & 1u) << b;
    iz |= int(oct & 1u) << b;
  }
}

}  // namespace fdm
