// Exclusive prefix sums and a stable LSD counting sort of (key, value) pairs
// on 4-bit digits: the Morton-keyed point ordering of the box trees.
#include "kernels.hpp"

namespace fdm {

namespace {

constexpr int kScanBlock = 256;
constexpr int kScanItems = 8;
constexpr int kScanTile = kScanBlock * kScanItems;

// Block-wide exclusive scan of one value per thread; returns the block total.
__device__ int64_t block_exclusive_scan(int64_t v, int64_t* shared, int64_t& total) {
  const int t = threadIdx.x;
  shared[t] = v;
  __syncthreads();
  for (int off = 1; off < kScanBlock; off <<= 1) {
    int64_t add = t >= off ? shared[t - off] : 0;
    __syncthreads();
    shared[t] += add;
    __syncthreads();
  }
  total = shared[kScanBlock - 1];
  int64_t excl = shared[t] - v;
  __syncthreads();
  return excl;
}

// Per tile: sum of the inputs.
__global__ void k_scan_reduce(const int32_t* in, int64_t n, int64_t* tile_sum) {
  __shared__ int64_t sh[kScanBlock];
  const int64_t base = int64_t(blockIdx.x) * kScanTile;
  int64_t s = 0;
  for (int i = 0; i < kScanItems; ++i) {
    int64_t j = base + int64_t(threadIdx.x) * kScanItems + i;
    if (j < n) s += in[j];
  }
  int64_t total;
  block_exclusive_scan(s, sh, total);
  if (threadIdx.x == 0) tile_sum[blockIdx.x] = total;
}

// Serial exclusive scan of the tile sums (few thousand entries at most).
__global__ void k_scan_tiles(int64_t* tile_sum, int64_t ntiles, int64_t* total) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  int64_t acc = 0;
  for (int64_t i = 0; i < ntiles; ++i) {
    int64_t v = tile_sum[i];
    tile_sum[i] = acc;
    acc += v;
  }
  *total = acc;
}

__global__ void k_scan_down(const int32_t* in, int64_t n, const int64_t* tile_off,
                            int32_t* out) {
  __shared__ int64_t sh[kScanBlock];
  const int64_t base = int64_t(blockIdx.x) * kScanTile;
  int64_t loc[kScanItems];
  int64_t s = 0;
  for (int i = 0; i < kScanItems; ++i) {
    int64_t j = base + int64_t(threadIdx.x) * kScanItems + i;
    loc[i] = s;
    if (j < n) s += in[j];
  }
  int64_t total;
  int64_t excl = block_exclusive_scan(s, sh, total);
  for (int i = 0; i < kScanItems; ++i) {
    int64_t j = base + int64_t(threadIdx.x) * kScanItems + i;
    if (j < n) out[j] = static_cast<int32_t>(tile_off[blockIdx.x] + excl + loc[i]);
  }
}

}  // namespace

int64_t exclusive_scan(const int32_t* in, int32_t* out, int64_t n,
                       hipStream_t s) {
  if (n == 0) return 0;
  int64_t ntiles = (n + kScanTile - 1) / kScanTile;
  DevBuf<int64_t> tiles(ntiles + 1);
  k_scan_reduce<<<ntiles, kScanBlock, 0, s>>>(in, n, tiles.get());
  FDM_LAUNCH("k_scan_reduce");
  k_scan_tiles<<<1, 64, 0, s>>>(tiles.get(), ntiles, tiles.get() + ntiles);
  FDM_LAUNCH("k_scan_tiles");
  k_scan_down<<<ntiles, kScanBlock, 0, s>>>(in, n, tiles.get(), out);
  FDM_LAUNCH("k_scan_down");
  int64_t total = 0;
  FDM_HIP(hipMemcpyAsync(&total, tiles.get() + ntiles, sizeof(int64_t),
                         hipMemcpyDeviceToHost, s));
  FDM_HIP(hipStreamSynchronize(s));
  return total;
}

namespace {

constexpr int kSortBlock = 256;
constexpr int kSortItems = 8;
constexpr int kSortTile = kSortBlock * kSortItems;
constexpr int kRadix = 16;

// Digit histogram of each tile: hist[digit * ntiles + tile].
__global__ void k_digit_hist(const uint32_t* keys, int64_t n, int shift,
                             int32_t* hist, int64_t ntiles) {
  __shared__ int32_t cnt[kRadix];
  if (threadIdx.x < kRadix) cnt[threadIdx.x] = 0;
  __syncthreads();
  const int64_t base = int64_t(blockIdx.x) * kSortTile;
  for (int i = 0; i < kSortItems; ++i) {
    int64_t j = base + int64_t(threadIdx.x) * kSortItems + i;
    if (j < n) atomicAdd(&cnt[(keys[j] >> shift) & (kRadix - 1)], 1);
  }
  __syncthreads();
  if (threadIdx.x < kRadix) hist[int64_t(threadIdx.x) * ntiles + blockIdx.x] = cnt[threadIdx.x];
}

// Stable scatter: the rank of an item is the scanned (digit, tile) offset,
// plus the items of the same digit held by lower threads of the tile, plus
// those earlier in the same thread (each thread holds consecutive items).
__global__ void k_digit_scatter(const uint32_t* keys, const int32_t* vals,
                                int64_t n, int shift, const int32_t* hist_off,
                                int64_t ntiles, uint32_t* keys_out,
                                int32_t* vals_out) {
  __shared__ int32_t cnt[kRadix][kSortBlock + 1];
  const int t = threadIdx.x;
  const int64_t base = int64_t(blockIdx.x) * kSortTile + int64_t(t) * kSortItems;
  uint32_t k[kSortItems];
  int32_t v[kSortItems];
  int d[kSortItems];
  int mine[kRadix];
  for (int r = 0; r < kRadix; ++r) mine[r] = 0;
  for (int i = 0; i < kSortItems; ++i) {
    int64_t j = base + i;
    if (j < n) {
      k[i] = keys[j];
      v[i] = vals[j];
      d[i] = (k[i] >> shift) & (kRadix - 1);
      for (int r = 0; r < kRadix; ++r) mine[r] += (d[i] == r);
    } else {
      d[i] = -1;
    }
  }
  for (int r = 0; r < kRadix; ++r) cnt[r][t] = mine[r];
  __syncthreads();
  // exclusive scan of cnt[r][0..255] for each digit r: 16 rows, 4 waves
  const int wave = t / 64, lane = t % 64;
  for (int r = wave; r < kRadix; r += kSortBlock / 64) {
    int a0 = cnt[r][4 * lane], a1 = cnt[r][4 * lane + 1],
        a2 = cnt[r][4 * lane + 2], a3 = cnt[r][4 * lane + 3];
    int s = a0 + a1 + a2 + a3;
    int incl = s;
    for (int off = 1; off < 64; off <<= 1) {
      int y = __shfl_up(incl, off, 64);
      if (lane >= off) incl += y;
    }
    int excl = incl - s;
    cnt[r][4 * lane] = excl;
    cnt[r][4 * lane + 1] = excl + a0;
    cnt[r][4 * lane + 2] = excl + a0 + a1;
    cnt[r][4 * lane + 3] = excl + a0 + a1 + a2;
  }
  __syncthreads();
  int seen[kRadix];
  for (int r = 0; r < kRadix; ++r) seen[r] = 0;
  for (int i = 0; i < kSortItems; ++i) {
    if (d[i] < 0) continue;
    int r = d[i];
    int sr = 0;
    for (int q = 0; q < kRadix; ++q) {
      sr += (q == r) ? seen[q] : 0;
      seen[q] += (q == r);
    }
    int64_t pos = int64_t(hist_off[int64_t(r) * ntiles + blockIdx.x]) + cnt[r][t] + sr;
    keys_out[pos] = k[i];
    vals_out[pos] = v[i];
  }
}

}  // namespace

void sort_pairs_stable(DevBuf<uint32_t>& keys, DevBuf<int32_t>& vals, int64_t n,
                       int key_bits, hipStream_t s) {
  if (n <= 1 || key_bits <= 0) return;
  int64_t ntiles = (n + kSortTile - 1) / kSortTile;
  DevBuf<uint32_t> k2(n);
  DevBuf<int32_t> v2(n);
  DevBuf<int32_t> hist(kRadix * ntiles), hoff(kRadix * ntiles);
  uint32_t *ka = keys.get(), *kb = k2.get();
  int32_t *va = vals.get(), *vb = v2.get();
  for (int shift = 0; shift < key_bits; shift += 4) {
    k_digit_hist<<<ntiles, kSortBlock, 0, s>>>(ka, n, shift, hist.get(), ntiles);
    FDM_LAUNCH("k_digit_hist");
    exclusive_scan(hist.get(), hoff.get(), kRadix * ntiles, s);
    k_digit_scatter<<<ntiles, kSortBlock, 0, s>>>(ka, va, n, shift, hoff.get(),
                                                  ntiles, kb, vb);
    FDM_LAUNCH("k_digit_scatter");
    std::swap(ka, kb);
    std::swap(va, vb);
  }
  if (ka != keys.get()) {
    FDM_HIP(hipMemcpyAsync(keys.get(), ka, n * sizeof(uint32_t), hipMemcpyDeviceToDevice, s));
    FDM_HIP(hipMemcpyAsync(vals.get(), va, n * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
  }
  FDM_HIP(hipStreamSynchronize(s));
}

}  // namespace fdm
