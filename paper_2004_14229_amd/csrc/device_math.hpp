// Device helpers: complex arithmetic, reduced-argument sincos, 1D Lagrange
// basis on Chebyshev nodes and the tensor-product transfer passes.
#pragma once

#include "kernels.hpp"

namespace fdm {

constexpr int kMaxK = kMaxM1 * kMaxM1 * kMaxM1;  // 729
constexpr int kPerLane = (kMaxK + 63) / 64;      // coefficients per lane
// Transfer kernels (M2M, L2L): one 256-thread workgroup per (box, direction)
// and the coefficients each thread holds.
constexpr int kXT = 256;
constexpr int kPerXT = (kMaxK + kXT - 1) / kXT;
// Dynamic LDS of the eight-children transfer kernels (k_m2m_oct, k_l2l_oct)
// at most: m <= 7; m = 8 takes the child-by-child kernels.
constexpr size_t kOctLds = 56 * 1024;

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// sin and cos of theta after reducing theta by 2*pi: k = rint(theta / 2pi),
// r = theta - k*C1 - k*C2 with C1 + C2 = 2*pi to about 106 bits, each step
// one fused multiply-add (Cody & Waite's additive reduction).
__device__ __forceinline__ void phase_sincos(double theta, double& s, double& c) {
  constexpr double kInv2Pi = 0.15915494309189533577;
  constexpr double kC1 = 6.283185307179586232;      // fl(2 pi)
  constexpr double kC2 = 2.4492935982947064e-16;    // 2 pi - fl(2 pi)
  const double k = rint(theta * kInv2Pi);
  double r = fma(-k, kC1, theta);
  r = fma(-k, kC2, r);
  sincos(r, &s, &c);
}

// l_nu(u) on the reference Chebyshev nodes of [-1, 1].
__device__ __forceinline__ double lagrange1d(const Interp& ip, int nu, double u) {
  double p = ip.wgt[nu];
  for (int mu = 0; mu < ip.m1; ++mu)
    if (mu != nu) p *= (u - ip.node[mu]);
  return p;
}

// One 1D pass of a tensor transfer along `axis` (0 = slowest index) for a
// (m+1)^3 complex array: out[.., j, ..] = sum_k W(j, k) in[.., k, ..] with
// W(j, k) = E1[b][j][k] (forward) or E1[b][k][j] (transposed).
__device__ __forceinline__ void transfer_pass(const double2* in, double2* out,
                                              const Interp& ip, int b, int axis,
                                              bool transposed, int lane, int nthreads) {
  const int m1 = ip.m1, K = ip.K;
  const int stride = axis == 0 ? m1 * m1 : axis == 1 ? m1 : 1;
  for (int e = lane; e < K; e += nthreads) {
    const int j = (e / stride) % m1;
    const int base = e - j * stride;
    double re = 0.0, im = 0.0;
    for (int k = 0; k < m1; ++k) {
      const double w = transposed ? ip.E1[b][k][j] : ip.E1[b][j][k];
      const double2 v = in[base + k * stride];
      re += w * v.x;
      im += w * v.y;
    }
    out[e] = make_double2(re, im);
  }
}

// buf[1] = E^T buf[0] (M2M) or E buf[0] (L2L) for the child octant bits bq;
// uses buf[0] as scratch.  Callers synchronise before and after.
__device__ __forceinline__ void apply_transfer(double2 (*buf)[kMaxK], const Interp& ip,
                                               const int bq[3], bool transposed,
                                               int lane, int nthreads) {
  transfer_pass(buf[0], buf[1], ip, bq[2], 2, transposed, lane, nthreads);
  __syncthreads();
  transfer_pass(buf[1], buf[0], ip, bq[1], 1, transposed, lane, nthreads);
  __syncthreads();
  transfer_pass(buf[0], buf[1], ip, bq[0], 0, transposed, lane, nthreads);
  __syncthreads();
}

}  // namespace fdm
