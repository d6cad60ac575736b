// Uniform box cluster trees on the GPU (Sect. 2.1, Alg. 1), refined to a
// fixed depth: every non-empty box above the leaf level is split at its
// centre c = (a + b)/2 into 8 half-open children, empty children dropped.
//
// A point's leaf is found by the same centre recursion per point (a point
// equal to a centre coordinate goes to the lower child); the octant path is
// its Morton key (x bit most significant).  Points are ordered by leaf key,
// ties by user index (stable counting sort); the boxes of a level are the
// distinct key prefixes, with a dense key -> box index grid per level.
#include "kernels.hpp"

namespace fdm {

namespace {

__global__ void k_leaf_keys(const double* __restrict__ pts, int64_t n,
                            double lo0, double lo1, double lo2, double hi0,
                            double hi1, double hi2, int levels,
                            uint32_t* __restrict__ keys, int32_t* __restrict__ idx,
                            int* __restrict__ outside) {
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * blockDim.x) {
    double p[3] = {pts[3 * i], pts[3 * i + 1], pts[3 * i + 2]};
    double lo[3] = {lo0, lo1, lo2};
    double hi[3] = {hi0, hi1, hi2};
    bool in = true;
    for (int d = 0; d < 3; ++d) in = in && (p[d] > lo[d]) && (p[d] <= hi[d]);
    uint32_t key = 0;
    if (!in) {
      atomicOr(outside, 1);
    } else {
      for (int l = 0; l < levels; ++l) {
        uint32_t oct = 0;
        for (int d = 0; d < 3; ++d) {
          double c = 0.5 * (lo[d] + hi[d]);
          bool up = p[d] > c;
          lo[d] = up ? c : lo[d];
          hi[d] = up ? hi[d] : c;
          oct = (oct << 1) | (up ? 1u : 0u);
        }
        key = (key << 3) | oct;
      }
    }
    keys[i] = key;
    idx[i] = static_cast<int32_t>(i);
  }
}

__global__ void k_gather_points(const double* __restrict__ pts,
                                const int32_t* __restrict__ idx, int64_t n,
                                double* x, double* y, double* z) {
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * blockDim.x) {
    int64_t j = idx[i];
    x[i] = pts[3 * j];
    y[i] = pts[3 * j + 1];
    z[i] = pts[3 * j + 2];
  }
}

__global__ void k_heads(const uint32_t* __restrict__ keys, int64_t n, int shift,
                        int32_t* __restrict__ head) {
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * blockDim.x)
    head[i] = (i == 0 || (keys[i] >> shift) != (keys[i - 1] >> shift)) ? 1 : 0;
}

__global__ void k_boxes(const uint32_t* __restrict__ keys, const int32_t* __restrict__ head,
                        const int32_t* __restrict__ pos, int64_t n, int shift,
                        uint32_t* __restrict__ bkey, int32_t* __restrict__ bstart,
                        int32_t* __restrict__ leaf_of) {
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * blockDim.x) {
    int32_t b = pos[i] + head[i] - 1;  // box of slot i
    if (head[i]) {
      bkey[b] = keys[i] >> shift;
      bstart[b] = static_cast<int32_t>(i);
    }
    if (leaf_of) leaf_of[i] = b;
  }
}

__global__ void k_counts(const int32_t* __restrict__ bstart, int64_t nb, int64_t n,
                         int32_t* __restrict__ bcount) {
  for (int64_t b = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; b < nb;
       b += int64_t(gridDim.x) * blockDim.x)
    bcount[b] = static_cast<int32_t>((b + 1 < nb ? bstart[b + 1] : n) - bstart[b]);
}

__global__ void k_fill_i32(int32_t* p, int64_t n, int32_t v) {
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * blockDim.x)
    p[i] = v;
}

__global__ void k_grid(const uint32_t* __restrict__ bkey, int64_t nb,
                       int32_t* __restrict__ grid) {
  for (int64_t b = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; b < nb;
       b += int64_t(gridDim.x) * blockDim.x)
    grid[bkey[b]] = static_cast<int32_t>(b);
}

}  // namespace

void build_tree(const double* pts_user, int64_t n, const double lo[3],
                const double hi[3], int levels, hipStream_t s, int64_t* tally,
                DevTree& T) {
  T.n = n;
  T.levels = levels;
  T.nb.assign(levels + 1, 0);
  T.key.resize(levels + 1);
  T.start.resize(levels + 1);
  T.count.resize(levels + 1);
  T.grid.resize(levels + 1);
  if (n == 0) return;
  const int B = 256;
  DevBuf<uint32_t> keys(n);
  DevBuf<int32_t> idx(n);
  DevBuf<int> outside(1);
  k_fill_i32<<<1, 64, 0, s>>>(outside.get(), 1, 0);
  k_leaf_keys<<<grid_for(n, B), B, 0, s>>>(pts_user, n, lo[0], lo[1], lo[2], hi[0],
                                           hi[1], hi[2], levels, keys.get(),
                                           idx.get(), outside.get());
  FDM_LAUNCH("k_leaf_keys");
  int out_flag = 0;
  FDM_HIP(hipMemcpyAsync(&out_flag, outside.get(), sizeof(int), hipMemcpyDeviceToHost, s));
  FDM_HIP(hipStreamSynchronize(s));
  if (out_flag)
    fail(FDM_ERR_POINT_OUTSIDE_BOX, "a point lies outside the root box (lo, hi]");

  sort_pairs_stable(keys, idx, n, 3 * levels, s);

  T.x.alloc(n, tally);
  T.y.alloc(n, tally);
  T.z.alloc(n, tally);
  k_gather_points<<<grid_for(n, B), B, 0, s>>>(pts_user, idx.get(), n, T.x.get(),
                                               T.y.get(), T.z.get());
  FDM_LAUNCH("k_gather_points");
  T.perm = std::move(idx);  // sorted user indices
  T.leaf_of.alloc(n, tally);

  DevBuf<int32_t> head(n), pos(n);
  for (int l = levels; l >= 0; --l) {
    int shift = 3 * (levels - l);
    k_heads<<<grid_for(n, B), B, 0, s>>>(keys.get(), n, shift, head.get());
    FDM_LAUNCH("k_heads");
    int64_t nb = exclusive_scan(head.get(), pos.get(), n, s);
    T.nb[l] = nb;
    T.key[l].alloc(nb, tally);
    T.start[l].alloc(nb, tally);
    T.count[l].alloc(nb, tally);
    k_boxes<<<grid_for(n, B), B, 0, s>>>(keys.get(), head.get(), pos.get(), n, shift,
                                         T.key[l].get(), T.start[l].get(),
                                         l == levels ? T.leaf_of.get() : nullptr);
    FDM_LAUNCH("k_boxes");
    k_counts<<<grid_for(nb, B), B, 0, s>>>(T.start[l].get(), nb, n, T.count[l].get());
    FDM_LAUNCH("k_counts");
    int64_t cells = int64_t(1) << (3 * l);
    T.grid[l].alloc(cells, tally);
    k_fill_i32<<<grid_for(cells, B), B, 0, s>>>(T.grid[l].get(), cells, -1);
    k_grid<<<grid_for(nb, B), B, 0, s>>>(T.key[l].get(), nb, T.grid[l].get());
    FDM_LAUNCH("k_grid");
  }
  FDM_HIP(hipStreamSynchronize(s));
}

void launch_fill_i32(int32_t* p, int64_t n, int32_t value, hipStream_t s) {
  if (n == 0) return;
  k_fill_i32<<<grid_for(n, 256), 256, 0, s>>>(p, n, value);
  FDM_LAUNCH("k_fill_i32");
}

}  // namespace fdm
