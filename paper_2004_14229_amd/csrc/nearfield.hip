// Near field of Alg. 4 (Sect. 2.6): y|_t += A|_{t x s} v|_s over the
// inadmissible leaf blocks, with A[j,k] = exp(i kappa r)/(4 pi r), r = |x_j - y_k|,
// evaluated directly in FP64 and zero for bitwise-equal points.  Also the
// dense product over all pairs (Sect. 1).
//
// The near-field blocks of a leaf are the same-level boxes at the leaf
// level's inadmissible offsets (independent of the target octant: an
// inadmissible pair always has an inadmissible, hence refined, parent).
// Small leaves (a few points each): one thread per target point in tree
// order, so neighbouring threads share a leaf and read the same source boxes
// (served from L2).  Large leaves (on average >= kLeafTile / 8 points): one
// workgroup per target leaf, each near source box staged through LDS in
// tiles that every thread of the leaf then reads (broadcast, no bank
// conflicts); both sum over the same offsets and sources in the same order,
// so they give the same bits.  The near field is stored into y (it runs
// before the far field, which is added).
#include "nearfield.hpp"

namespace fdm {

namespace {

// Thread per target point (stores the near field into y).
__global__ void __launch_bounds__(256) k_p2p(P2PDesc d, int64_t nT) {
  const int64_t j = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  if (j >= nT) return;
  reinterpret_cast<double2*>(d.y)[j] = near_value(d, j);
}

// Workgroup per target leaf (grid-stride), its points kLeafTile at a time.
constexpr int kLeafTile = 256;
__global__ void __launch_bounds__(kLeafTile) k_p2p_leaf(P2PDesc d,
                                                        const int32_t* __restrict__ startT,
                                                        const int32_t* __restrict__ countT,
                                                        int64_t n_leaf) {
  __shared__ double sx[kLeafTile], sy[kLeafTile], sz[kLeafTile];
  __shared__ double2 sv[kLeafTile];
  const double2* v = reinterpret_cast<const double2*>(d.v);
  const int lim = 1 << d.level;
  for (int64_t b = blockIdx.x; b < n_leaf; b += gridDim.x) {
    int ix, iy, iz;
    demorton3(d.keyT[b], d.level, ix, iy, iz);
    const int t0 = startT[b], tn = countT[b];
    for (int tb = 0; tb < tn; tb += kLeafTile) {
      const int j = t0 + tb + threadIdx.x;
      const bool act = tb + static_cast<int>(threadIdx.x) < tn;
      double px = 0.0, py = 0.0, pz = 0.0;
      if (act) {
        px = d.xt[j];
        py = d.yt[j];
        pz = d.zt[j];
      }
      double ar = 0.0, ai = 0.0;
      for (int o = 0; o < d.n_off; ++o) {
        const int sxb = ix - d.near_off[3 * o], syb = iy - d.near_off[3 * o + 1],
                  szb = iz - d.near_off[3 * o + 2];
        if (sxb < 0 || syb < 0 || szb < 0 || sxb >= lim || syb >= lim || szb >= lim) continue;
        const int32_t sb = d.gridS[morton3(sxb, syb, szb, d.level)];
        if (sb < 0) continue;
        const int k0 = d.startS[sb], kn = d.countS[sb];
        for (int kb = 0; kb < kn; kb += kLeafTile) {
          __syncthreads();  // the previous tile has been read
          const int k = kb + static_cast<int>(threadIdx.x);
          if (k < kn) {
            sx[threadIdx.x] = d.xs[k0 + k];
            sy[threadIdx.x] = d.ys[k0 + k];
            sz[threadIdx.x] = d.zs[k0 + k];
            sv[threadIdx.x] = v[k0 + k];
          }
          __syncthreads();
          const int nk = kn - kb < kLeafTile ? kn - kb : kLeafTile;
          if (act)
            for (int q = 0; q < nk; ++q)
              kernel_add(px, py, pz, sx[q], sy[q], sz[q], sv[q], d.kappa, ar, ai);
        }
      }
      if (act) reinterpret_cast<double2*>(d.y)[j] = make_double2(ar, ai);
    }
  }
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

P2PDesc p2p_desc(const Plan& P) {
  const int p = P.levels;
  P2PDesc d{};
  d.xt = P.T.x.get();
  d.yt = P.T.y.get();
  d.zt = P.T.z.get();
  d.leaf_of = P.T.leaf_of.get();
  d.keyT = P.T.key[p].get();
  d.xs = P.S.x.get();
  d.ys = P.S.y.get();
  d.zs = P.S.z.get();
  d.v = P.vtree();
  d.startS = P.S.start[p].get();
  d.countS = P.S.count[p].get();
  d.gridS = P.S.grid[p].get();
  d.near_off = P.near_off.get();
  d.y = P.ytree();
  d.kappa = P.kappa;
  d.n_off = P.n_near_off;
  d.level = p;
  return d;
}

void launch_p2p(Plan& P, hipStream_t s) {
  if (P.nT == 0 || P.nS == 0) return;
  if (P.adaptive()) {
    launch_p2p_adaptive(P, s);
    return;
  }
  const int p = P.levels;
  const int64_t n_leaf = P.T.nb[p];
  if (n_leaf > 0 && P.nT >= int64_t(kLeafTile / 8) * n_leaf) {  // large leaves
    const unsigned grid = static_cast<unsigned>(std::min<int64_t>(n_leaf, 1 << 20));
    k_p2p_leaf<<<grid, kLeafTile, 0, s>>>(p2p_desc(P), P.T.start[p].get(), P.T.count[p].get(),
                                          n_leaf);
    FDM_LAUNCH("k_p2p_leaf");
    return;
  }
  const int B = 256;
  k_p2p<<<static_cast<unsigned>((P.nT + B - 1) / B), B, 0, s>>>(p2p_desc(P), P.nT);
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
