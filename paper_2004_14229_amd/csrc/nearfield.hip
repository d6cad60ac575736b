// Near field of Alg. 4 (Sect. 2.6): y|_t += A|_{t x s} v|_s over the
// inadmissible leaf blocks, with A[j,k] = exp(i kappa r)/(4 pi r), r = |x_j - y_k|,
// evaluated directly in FP64 and zero for bitwise-equal points.  Also the
// dense product over all pairs (Sect. 1).
//
// The near-field blocks of a leaf are the same-level boxes at the leaf
// level's inadmissible offsets (independent of the target octant: an
// inadmissible pair always has an inadmissible, hence refined, parent).
// One thread per target point in tree order, so neighbouring threads share
// a leaf and read the same source boxes (served from L2).
#include "plan.hpp"
#include "device_math.hpp"

namespace fdm {

namespace {

__device__ __forceinline__ void kernel_add(double xt, double yt, double zt, double xs,
                                           double ys, double zs, double2 v, double kappa,
                                           double& ar, double& ai) {
  const double dx = xt - xs, dy = yt - ys, dz = zt - zs;
  if (xt == xs && yt == ys && zt == zs) return;  // f(x, x) = 0
  const double r = sqrt(dx * dx + dy * dy + dz * dz);
  double sn, cs;
  phase_sincos(kappa * r, sn, cs);
  const double w = 1.0 / (4.0 * M_PI * r);
  const double fr = cs * w, fi = sn * w;
  ar += fr * v.x - fi * v.y;
  ai += fr * v.y + fi * v.x;
}

// Thread per target point: loop over the near offsets of its leaf.
__global__ void __launch_bounds__(256) k_p2p(
    const double* __restrict__ xt, const double* __restrict__ yt,
    const double* __restrict__ zt, const int32_t* __restrict__ leaf_of, int64_t nT,
    const uint32_t* __restrict__ keyT, const double* __restrict__ xs,
    const double* __restrict__ ys, const double* __restrict__ zs,
    const double2* __restrict__ v, const int32_t* __restrict__ startS,
    const int32_t* __restrict__ countS, const int32_t* __restrict__ gridS,
    const int32_t* __restrict__ near_off, int n_off, int level, double kappa,
    double2* __restrict__ y_tree) {
  const int64_t j = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  if (j >= nT) return;
  const double px = xt[j], py = yt[j], pz = zt[j];
  int ix, iy, iz;
  demorton3(keyT[leaf_of[j]], level, ix, iy, iz);
  const int lim = 1 << level;
  double ar = 0.0, ai = 0.0;
  for (int o = 0; o < n_off; ++o) {
    const int sx = ix - near_off[3 * o], sy = iy - near_off[3 * o + 1],
              sz = iz - near_off[3 * o + 2];
    if (sx < 0 || sy < 0 || sz < 0 || sx >= lim || sy >= lim || sz >= lim) continue;
    const int32_t sb = gridS[morton3(sx, sy, sz, level)];
    if (sb < 0) continue;
    const int k0 = startS[sb], kn = countS[sb];
    for (int k = k0; k < k0 + kn; ++k)
      kernel_add(px, py, pz, xs[k], ys[k], zs[k], v[k], kappa, ar, ai);
  }
  const double2 prev = y_tree[j];
  y_tree[j] = make_double2(prev.x + ar, prev.y + ai);
}

// Dense product: thread per target, source tiles staged in LDS.
constexpr int kDenseTile = 256;
__global__ void __launch_bounds__(kDenseTile) k_dense(
    const double* __restrict__ pT, int64_t nT, const double* __restrict__ pS, int64_t nS,
    double kappa, const double2* __restrict__ v, double2* __restrict__ y) {
  __shared__ double sx[kDenseTile], sy[kDenseTile], sz[kDenseTile];
  __shared__ double2 sv[kDenseTile];
  const int64_t j = blockIdx.x * int64_t(kDenseTile) + threadIdx.x;
  const bool act = j < nT;
  double px = 0, py = 0, pz = 0;
  if (act) {
    px = pT[3 * j];
    py = pT[3 * j + 1];
    pz = pT[3 * j + 2];
  }
  double ar = 0.0, ai = 0.0;
  for (int64_t t0 = 0; t0 < nS; t0 += kDenseTile) {
    const int64_t k = t0 + threadIdx.x;
    __syncthreads();
    if (k < nS) {
      sx[threadIdx.x] = pS[3 * k];
      sy[threadIdx.x] = pS[3 * k + 1];
      sz[threadIdx.x] = pS[3 * k + 2];
      sv[threadIdx.x] = v[k];
    }
    __syncthreads();
    const int nk = static_cast<int>(nS - t0 < kDenseTile ? nS - t0 : kDenseTile);
    if (act)
      for (int q = 0; q < nk; ++q)
        kernel_add(px, py, pz, sx[q], sy[q], sz[q], sv[q], kappa, ar, ai);
  }
  if (act) y[j] = make_double2(ar, ai);
}

}  // namespace

void launch_p2p(Plan& P, hipStream_t s) {
  const int p = P.levels;
  if (P.nT == 0 || P.nS == 0 || P.n_near_off == 0) return;
  const int B = 256;
  k_p2p<<<static_cast<unsigned>((P.nT + B - 1) / B), B, 0, s>>>(
      P.T.x.get(), P.T.y.get(), P.T.z.get(), P.T.leaf_of.get(), P.nT, P.T.key[p].get(),
      P.S.x.get(), P.S.y.get(), P.S.z.get(), reinterpret_cast<const double2*>(P.v_tree.get()),
      P.S.start[p].get(), P.S.count[p].get(), P.S.grid[p].get(), P.near_off.get(),
      P.n_near_off, p, P.kappa, reinterpret_cast<double2*>(P.y_tree.get()));
  FDM_LAUNCH("k_p2p");
}

void launch_dense(const double* pT, int64_t nT, const double* pS, int64_t nS, double kappa,
                  const double* v, double* y, hipStream_t s) {
  if (nT == 0) return;
  k_dense<<<static_cast<unsigned>((nT + kDenseTile - 1) / kDenseTile), kDenseTile, 0, s>>>(
      pT, nT, pS, nS, kappa, reinterpret_cast<const double2*>(v), reinterpret_cast<double2*>(y));
  FDM_LAUNCH("k_dense");
}

}  // namespace fdm
