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
// without the pruned boxes; S2M and L2T run over per-level leaf lists; the
// near-field blocks of each target box are listed at plan build.
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

constexpr int kNearThreads = 256;

// One workgroup per near-field item: the sums over the item's blocks for
// each of its target points, stored into z[level * nT + point].  Sources are
// staged through LDS in tiles of 256; an item of n <= 128 points gives each
// point 256 / 2^ceil(log2 n) lanes, each taking every such source of a tile,
// and their partial sums are added in lane order.
__global__ void __launch_bounds__(kNearThreads) k_near_items(
    const int4* __restrict__ items, const int2* __restrict__ ranges,
    const double* __restrict__ xt, const double* __restrict__ yt,
    const double* __restrict__ zt, const double* __restrict__ xs,
    const double* __restrict__ ys, const double* __restrict__ zs,
    const double2* __restrict__ v, double kappa, double2* __restrict__ z, int64_t nT) {
  __shared__ int32_t pre[kNearThreads + 1];  // exclusive prefix of the batch's counts
  __shared__ int32_t rst[kNearThreads];      // first source slot of each range
  __shared__ double sx[kNearThreads], sy[kNearThreads], sz[kNearThreads];
  __shared__ double2 sv[kNearThreads];
  const int t = threadIdx.x;
  const int4 it = items[blockIdx.x];
  const int n = it.y & 0xffff, level = it.y >> 16;
  int pw = 1;
  while (pw < n) pw <<= 1;
  const int sub = kNearThreads / pw;
  const int i = t / sub, q = t % sub;
  const bool act = i < n;
  double px = 0.0, py = 0.0, pz = 0.0;
  if (act) {
    px = xt[it.x + i];
    py = yt[it.x + i];
    pz = zt[it.x + i];
  }
  double ar = 0.0, ai = 0.0;
  for (int rb = it.z; rb < it.w; rb += kNearThreads) {
    const int nr = min(kNearThreads, it.w - rb);
    int c = 0;
    if (t < nr) {
      const int2 r = ranges[rb + t];
      rst[t] = r.x;
      c = r.y;
    }
    pre[t + 1] = c;
    if (t == 0) pre[0] = 0;
    __syncthreads();
    for (int off = 1; off < kNearThreads; off <<= 1) {  // inclusive scan of pre[1..]
      const int x = t >= off ? pre[t + 1 - off] : 0;
      __syncthreads();
      pre[t + 1] += x;
      __syncthreads();
    }
    const int total = pre[nr];
    for (int s0 = 0; s0 < total; s0 += kNearThreads) {
      const int g = s0 + t;
      if (g < total) {  // the range holding flat index g: last r with pre[r] <= g
        int lo = 0, hi = nr - 1;
        while (lo < hi) {
          const int mid = (lo + hi + 1) >> 1;
          if (pre[mid] <= g) lo = mid; else hi = mid - 1;
        }
        const int k = rst[lo] + (g - pre[lo]);
        sx[t] = xs[k];
        sy[t] = ys[k];
        sz[t] = zs[k];
        sv[t] = v[k];
      }
      __syncthreads();
      const int tile = min(kNearThreads, total - s0);
      if (act)
        for (int u = q; u < tile; u += sub)
          kernel_add(px, py, pz, sx[u], sy[u], sz[u], sv[u], kappa, ar, ai);
      __syncthreads();
    }
    __syncthreads();  // the batch's prefix and starts are read up to here
  }
  sv[t] = make_double2(ar, ai);
  __syncthreads();
  if (act && q == 0) {
    double2 acc = sv[t];
    for (int u = 1; u < sub; ++u) {
      acc.x += sv[t + u].x;
      acc.y += sv[t + u].y;
    }
    z[int64_t(level) * nT + it.x + i] = acc;
  }
}

// y[j] = the sum of point j's level sums, from the root to its leaf.
__global__ void k_near_sum(const double2* __restrict__ z, const uint8_t* __restrict__ leaf_level,
                           int64_t nT, double2* __restrict__ y) {
  const int64_t j = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  if (j >= nT) return;
  double ar = 0.0, ai = 0.0;
  for (int l = 0; l <= leaf_level[j]; ++l) {
    const double2 a = z[l * nT + j];
    ar += a.x;
    ai += a.y;
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
  FDM_HIP(hipStreamSynchronize(s));
}

// The near-field blocks of every existing target box, level by level (the
// pairs (t, s) at the level's inadmissible offsets whose t or s is a leaf),
// as source point ranges in work items of at most 256 target points, most
// work first, and the near-field statistics.
void adaptive_near_field(Plan& P, hipStream_t s) {
  const int p = P.levels;
  P.near_pairs = 0;
  P.near_entries = 0;
  std::vector<int2> ranges;
  std::vector<std::pair<int64_t, int4>> items;  // (work, item)
  std::vector<uint8_t> leaf_level(P.nT, 0);
  for (int l = 0; l <= p; ++l) {
    std::vector<uint32_t> kT = to_host(P.T.key[l].get(), P.T.nb[l], s);
    std::vector<int32_t> sT = to_host(P.T.start[l].get(), P.T.nb[l], s);
    std::vector<int32_t> cT = to_host(P.T.count[l].get(), P.T.nb[l], s);
    std::vector<int32_t> gS = to_host(P.gridS_alive[l].get(), size_t(1) << (3 * l), s);
    std::vector<int32_t> sS = to_host(P.S.start[l].get(), P.S.nb[l], s);
    std::vector<int32_t> cS = to_host(P.S.count[l].get(), P.S.nb[l], s);
    const int lim = 1 << l;
    for (size_t b = 0; b < kT.size(); ++b) {
      const uint8_t st = P.stateT_h[l][b];
      if (st == 0) continue;
      if (st == 2) std::fill_n(leaf_level.begin() + sT[b], cT[b], static_cast<uint8_t>(l));
      const size_t r0 = ranges.size();
      int64_t ns = 0;
      int ix, iy, iz;
      demorton3(kT[b], l, ix, iy, iz);
      for (const Off& o : P.tab[l].inadm) {
        if (P.nS == 0) break;
        const int sx = ix - o.x, sy = iy - o.y, sz = iz - o.z;
        if (sx < 0 || sy < 0 || sz < 0 || sx >= lim || sy >= lim || sz >= lim) continue;
        const int32_t sb = gS[morton3(sx, sy, sz, l)];
        if (sb < 0) continue;
        if (st != 2 && P.stateS_h[l][sb] != 2) continue;  // refined pair
        ranges.push_back(make_int2(sS[sb], cS[sb]));
        ns += cS[sb];
        ++P.near_pairs;
        P.near_entries += int64_t(cT[b]) * cS[sb];
      }
      if (ranges.size() > size_t(INT32_MAX)) fail(FDM_ERR_UNSUPPORTED, "near-field lists too long");
      for (int32_t c = 0; c < cT[b]; c += kNearThreads) {
        const int32_t n = std::min(kNearThreads, cT[b] - c);
        items.push_back({int64_t(n) * ns + n,
                         make_int4(sT[b] + c, n | (l << 16), static_cast<int32_t>(r0),
                                   static_cast<int32_t>(ranges.size()))});
      }
    }
  }
  std::stable_sort(items.begin(), items.end(),
                   [](const auto& a, const auto& b) { return a.first > b.first; });
  std::vector<int4> it(items.size());
  for (size_t k = 0; k < items.size(); ++k) it[k] = items[k].second;
  P.n_near_items = static_cast<int64_t>(it.size());
  to_device(P.near_items, it, s, &P.tally);
  to_device(P.near_ranges, ranges, s, &P.tally);
  to_device(P.near_leaf_level, leaf_level, s, &P.tally);
  P.near_z.alloc(size_t(2) * (p + 1) * P.nT, &P.tally);
  FDM_HIP(hipStreamSynchronize(s));
}

// Every item writes its points' sums of its level, and every point lies in
// one item of each level from the root to its leaf, so the level sums are
// complete without clearing.
void launch_p2p_adaptive(Plan& P, hipStream_t s) {
  if (P.nT == 0) return;
  double2* z = reinterpret_cast<double2*>(P.near_z.get());
  if (P.n_near_items) {
    k_near_items<<<static_cast<unsigned>(P.n_near_items), kNearThreads, 0, s>>>(
        P.near_items.get(), P.near_ranges.get(), P.T.x.get(), P.T.y.get(), P.T.z.get(),
        P.S.x.get(), P.S.y.get(), P.S.z.get(), reinterpret_cast<const double2*>(P.vtree()),
        P.kappa, z, P.nT);
    FDM_LAUNCH("k_near_items");
  }
  k_near_sum<<<grid_for(P.nT, 256), 256, 0, s>>>(z, P.near_leaf_level.get(), P.nT,
                                                  reinterpret_cast<double2*>(P.ytree()));
  FDM_LAUNCH("k_near_sum");
}

}  // namespace fdm
