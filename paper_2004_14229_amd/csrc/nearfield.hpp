// Near field of Alg. 4 (Sect. 2.6) for one target point: the sum of
// A[j,k] v_k over the source points of the inadmissible leaf blocks of its
// leaf, A[j,k] = exp(i kappa r)/(4 pi r), r = |x_j - y_k|, evaluated directly
// in FP64 and zero for bitwise-equal points.
#pragma once

#include "plan.hpp"
#include "device_math.hpp"

namespace fdm {

// f(x, y) as (fr, fi); false (and f = 0) for bitwise-equal points.
__device__ __forceinline__ bool kernel_value(double xt, double yt, double zt, double xs,
                                             double ys, double zs, double kappa, double& fr,
                                             double& fi) {
  const double dx = xt - xs, dy = yt - ys, dz = zt - zs;
  if (xt == xs && yt == ys && zt == zs) return false;  // f(x, x) = 0
  const double r = sqrt(dx * dx + dy * dy + dz * dz);
  double sn, cs;
  phase_sincos(kappa * r, sn, cs);
  const double w = 1.0 / (4.0 * M_PI * r);
  fr = cs * w;
  fi = sn * w;
  return true;
}

// (ar, ai) += f v as four fused multiply-adds in a fixed order, so that every
// kernel that sums near-field terms rounds them the same way.
__device__ __forceinline__ void kernel_accumulate(double fr, double fi, double2 v, double& ar,
                                                  double& ai) {
  ar = fma(fr, v.x, ar);
  ar = fma(-fi, v.y, ar);
  ai = fma(fr, v.y, ai);
  ai = fma(fi, v.x, ai);
}

__device__ __forceinline__ void kernel_add(double xt, double yt, double zt, double xs,
                                           double ys, double zs, double2 v, double kappa,
                                           double& ar, double& ai) {
  double fr, fi;
  if (!kernel_value(xt, yt, zt, xs, ys, zs, kappa, fr, fi)) return;
  kernel_accumulate(fr, fi, v, ar, ai);
}

// Near-field value of target point j (tree order); the near-field blocks of
// a leaf are the same-level boxes at the leaf level's inadmissible offsets.
__device__ __forceinline__ double2 near_value(const P2PDesc& d, int64_t j) {
  const double px = d.xt[j], py = d.yt[j], pz = d.zt[j];
  int ix, iy, iz;
  demorton3(d.keyT[d.leaf_of[j]], d.level, ix, iy, iz);
  const int lim = 1 << d.level;
  const double2* v = reinterpret_cast<const double2*>(d.v);
  double ar = 0.0, ai = 0.0;
  for (int o = 0; o < d.n_off; ++o) {
    const int sx = ix - d.near_off[3 * o], sy = iy - d.near_off[3 * o + 1],
              sz = iz - d.near_off[3 * o + 2];
    if (sx < 0 || sy < 0 || sz < 0 || sx >= lim || sy >= lim || sz >= lim) continue;
    const int32_t sb = d.gridS[morton3(sx, sy, sz, d.level)];
    if (sb < 0) continue;
    const int k0 = d.startS[sb], kn = d.countS[sb];
    for (int k = k0; k < k0 + kn; ++k)
      kernel_add(px, py, pz, d.xs[k], d.ys[k], d.zs[k], v[k], d.kappa, ar, ai);
  }
  return make_double2(ar, ai);
}

}  // namespace fdm
