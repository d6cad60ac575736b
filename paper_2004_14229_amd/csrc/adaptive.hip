// Adaptive box cluster trees (Sect. 2.1, Alg. 1 with its n_max stop rule)
// on top of the full-depth device trees.
//
// Alg. 1 refines a box while it holds more than n_max points (here also at
// most down to the plan's depth).  The device trees are refined to the full
// depth; a box of level l exists in the adaptive tree when its parent
// exists and was refined, i.e. holds more than n_max points and lies above
// the last level.  Per level and box the state is 0 (pruned), 1 (refined)
// or 2 (leaf).
//
// What changes in Alg. 2 and Alg. 4 (Sect. 2.3, 2.6):
//  * a pair (t, s) of one level is a block when both boxes exist and the
//    parent offset was inadmissible (as for uniform trees); admissible
//    blocks are couplings whatever the boxes' states, and an inadmissible
//    block with a leaf on either side is a near-field block, on any level;
//  * moments of a leaf of any level come from its own points (S2M), those
//    of a refined box from its children (M2M); the far field of a target
//    leaf of any level is evaluated from its locals (L2T).
// The coupling items run over existing target boxes against a source grid
// without the pruned boxes; S2M and L2T run over per-level leaf lists.
#include <algorithm>

#include "plan.hpp"
#include "nearfield.hpp"

namespace fdm {

namespace {

__global__ void k_prune_grid(const uint32_t* __restrict__ key, const uint8_t* __restrict__ state,
                             int64_t nb, int32_t* __restrict__ grid) {
  for (int64_t b = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; b < nb;
       b += int64_t(gridDim.x) * blockDim.x)
    if (state[b] == 0) grid[key[b]] = -1;
}

// Thread per target point (tree order): the near-field blocks of its boxes
// on every level down to its leaf, stored into y.  On level l its box t
// meets the existing source boxes s = t - o at the level's inadmissible
// offsets o; the pair is a near-field block when t is a leaf or s is.
__global__ void __launch_bounds__(256) k_p2p_adaptive(
    const AdaptNear* __restrict__ lv, int p, const uint32_t* __restrict__ keyTp,
    const int32_t* __restrict__ leaf_of, const double* __restrict__ xt,
    const double* __restrict__ yt, const double* __restrict__ zt,
    const double* __restrict__ xs, const double* __restrict__ ys,
    const double* __restrict__ zs, const double2* __restrict__ v,
    const int32_t* __restrict__ off, const int32_t* __restrict__ off_begin, double kappa,
    double2* __restrict__ y, int64_t nT) {
  const int64_t j = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  if (j >= nT) return;
  const double px = xt[j], py = yt[j], pz = zt[j];
  const uint32_t kp = keyTp[leaf_of[j]];
  double ar = 0.0, ai = 0.0;
  for (int l = 0; l <= p; ++l) {
    const AdaptNear L = lv[l];
    const uint32_t kl = kp >> (3 * (p - l));
    const int32_t tb = L.gridT[kl];
    const bool leafT = L.stateT[tb] == 2;
    int ix, iy, iz;
    demorton3(kl, l, ix, iy, iz);
    const int lim = 1 << l;
    for (int i = off_begin[l]; i < off_begin[l + 1]; ++i) {
      const int sx = ix - off[3 * i], sy = iy - off[3 * i + 1], sz = iz - off[3 * i + 2];
      if (sx < 0 || sy < 0 || sz < 0 || sx >= lim || sy >= lim || sz >= lim) continue;
      const int32_t sb = L.gridS[morton3(sx, sy, sz, l)];
      if (sb < 0) continue;
      if (!leafT && L.stateS[sb] != 2) continue;  // refined pair: not a leaf block
      const int k0 = L.startS[sb], kn = L.countS[sb];
      for (int k = k0; k < k0 + kn; ++k)
        kernel_add(px, py, pz, xs[k], ys[k], zs[k], v[k], kappa, ar, ai);
    }
    if (leafT) break;
  }
  y[j] = make_double2(ar, ai);
}

// States of one tree's boxes, level by level, from the box counts.
std::vector<std::vector<uint8_t>> tree_states(const DevTree& A, int p, int64_t n_max,
                                              hipStream_t s) {
  std::vector<std::vector<uint8_t>> st(p + 1);
  std::vector<uint32_t> kprev;
  for (int l = 0; l <= p; ++l) {
    const int64_t nb = A.nb[l];
    std::vector<uint32_t> keys = to_host(A.key[l].get(), nb, s);
    std::vector<int32_t> cnt = to_host(A.count[l].get(), nb, s);
    st[l].assign(nb, 0);
    for (int64_t b = 0; b < nb; ++b) {
      bool exists = l == 0;
      if (l > 0) {
        const uint32_t pk = keys[b] >> 3;
        const auto it = std::lower_bound(kprev.begin(), kprev.end(), pk);
        exists = it != kprev.end() && *it == pk && st[l - 1][it - kprev.begin()] == 1;
      }
      if (exists) st[l][b] = (l == p || cnt[b] <= n_max) ? 2 : 1;
    }
    kprev.swap(keys);
  }
  return st;
}

std::vector<int32_t> leaves_of(const std::vector<uint8_t>& st) {
  std::vector<int32_t> out;
  for (size_t b = 0; b < st.size(); ++b)
    if (st[b] == 2) out.push_back(static_cast<int32_t>(b));
  return out;
}

}  // namespace

void build_adaptive(Plan& P, hipStream_t s) {
  const int p = P.levels;
  P.stateT_h = tree_states(P.T, p, P.n_max, s);
  P.stateS_h = tree_states(P.S, p, P.n_max, s);
  P.stateT.clear();
  P.stateS.clear();
  P.gridS_alive.clear();
  P.leafT.clear();
  P.leafS.clear();
  P.stateT.resize(p + 1);
  P.stateS.resize(p + 1);
  P.gridS_alive.resize(p + 1);
  P.leafT.resize(p + 1);
  P.leafS.resize(p + 1);
  P.n_leafT.assign(p + 1, 0);
  P.n_leafS.assign(p + 1, 0);
  for (int l = 0; l <= p; ++l) {
    to_device(P.stateT[l], P.stateT_h[l], s, &P.tally);
    to_device(P.stateS[l], P.stateS_h[l], s, &P.tally);
    const std::vector<int32_t> lt = leaves_of(P.stateT_h[l]), ls = leaves_of(P.stateS_h[l]);
    to_device(P.leafT[l], lt, s, &P.tally);
    to_device(P.leafS[l], ls, s, &P.tally);
    P.n_leafT[l] = static_cast<int64_t>(lt.size());
    P.n_leafS[l] = static_cast<int64_t>(ls.size());
    const size_t cells = size_t(1) << (3 * l);
    P.gridS_alive[l].alloc(cells, &P.tally);
    FDM_HIP(hipMemcpyAsync(P.gridS_alive[l].get(), P.S.grid[l].get(), cells * sizeof(int32_t),
                           hipMemcpyDeviceToDevice, s));
    if (P.S.nb[l]) {
      k_prune_grid<<<grid_for(P.S.nb[l], 256), 256, 0, s>>>(
          P.S.key[l].get(), P.stateS[l].get(), P.S.nb[l], P.gridS_alive[l].get());
      FDM_LAUNCH("k_prune_grid");
    }
  }
  // inadmissible offsets of every level, for the near field
  std::vector<int32_t> off;
  P.adapt_off_begin.assign(1, 0);
  for (int l = 0; l <= p; ++l) {
    for (const Off& o : P.tab[l].inadm) off.insert(off.end(), {o.x, o.y, o.z});
    P.adapt_off_begin.push_back(static_cast<int32_t>(off.size() / 3));
  }
  to_device(P.adapt_off, off, s, &P.tally);
  to_device(P.adapt_off_begin_d, P.adapt_off_begin, s, &P.tally);
  std::vector<AdaptNear> lv(p + 1);
  for (int l = 0; l <= p; ++l)
    lv[l] = AdaptNear{P.T.grid[l].get(), P.stateT[l].get(), P.gridS_alive[l].get(),
                      P.stateS[l].get(), P.S.start[l].get(), P.S.count[l].get()};
  to_device(P.adapt_near, lv, s, &P.tally);
  FDM_HIP(hipStreamSynchronize(s));
}

void adaptive_near_stats(Plan& P, hipStream_t s) {
  P.near_pairs = 0;
  P.near_entries = 0;
  if (P.nT == 0 || P.nS == 0) return;
  for (int l = 0; l <= P.levels; ++l) {
    std::vector<uint32_t> kT = to_host(P.T.key[l].get(), P.T.nb[l], s);
    std::vector<int32_t> cT = to_host(P.T.count[l].get(), P.T.nb[l], s);
    std::vector<int32_t> gS = to_host(P.gridS_alive[l].get(), size_t(1) << (3 * l), s);
    std::vector<int32_t> cS = to_host(P.S.count[l].get(), P.S.nb[l], s);
    const int lim = 1 << l;
    for (size_t b = 0; b < kT.size(); ++b) {
      const uint8_t st = P.stateT_h[l][b];
      if (st == 0) continue;
      int ix, iy, iz;
      demorton3(kT[b], l, ix, iy, iz);
      for (const Off& o : P.tab[l].inadm) {
        const int sx = ix - o.x, sy = iy - o.y, sz = iz - o.z;
        if (sx < 0 || sy < 0 || sz < 0 || sx >= lim || sy >= lim || sz >= lim) continue;
        const int32_t sb = gS[morton3(sx, sy, sz, l)];
        if (sb < 0) continue;
        if (st != 2 && P.stateS_h[l][sb] != 2) continue;
        ++P.near_pairs;
        P.near_entries += int64_t(cT[b]) * cS[sb];
      }
    }
  }
}

void launch_p2p_adaptive(Plan& P, hipStream_t s) {
  if (P.nT == 0 || P.nS == 0) return;
  const int B = 256;
  k_p2p_adaptive<<<static_cast<unsigned>((P.nT + B - 1) / B), B, 0, s>>>(
      P.adapt_near.get(), P.levels, P.T.key[P.levels].get(), P.T.leaf_of.get(), P.T.x.get(),
      P.T.y.get(), P.T.z.get(), P.S.x.get(), P.S.y.get(), P.S.z.get(),
      reinterpret_cast<const double2*>(P.vtree()), P.adapt_off.get(),
      P.adapt_off_begin_d.get(), P.kappa, reinterpret_cast<double2*>(P.ytree()), P.nT);
  FDM_LAUNCH("k_p2p_adaptive");
}

}  // namespace fdm
