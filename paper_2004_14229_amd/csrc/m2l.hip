// Coupling step of Alg. 4 (Sect. 2.6, M2L): g~_{t,c} = sum_s A~_{c,t x s} v~_{s,c}
// over the admissible blocks, on the matrix cores.
//
// Bank (Sect. 2.7): the coupling matrix of a block depends only on its level
// and offset o = i_t - i_s, so one K x K complex matrix is needed per
// admissible (level, offset):
//   A~[j,k] = f(xi_{t,j}, xi_{s,k}) exp(-i kappa <(xi_{t,j}-m_t) - (xi_{s,k}-m_s), c>)
// (the paper's f_c with the plane-wave factors of the box centres moved into
// the moments and locals), evaluated in FP64 and stored as split re/im
// planes, transposed (k-major) so that a wave's rows of one k are contiguous
// (FP64, FP32), or as BF16 hi/lo planes in MFMA operand order.  The bank is
// either resident or generated, a range of matrices at a time, into a
// workspace right before the items that use it.
//
// Product: one work item is a block of up to nb (32 or 64) target boxes of
// one level, one octant (so they share the list of admissible offsets) and
// one direction c.  Its workgroup loops over that list's offsets that hit
// at least one non-empty source box, gathers the source moment columns
// t - o (zero for missing boxes) through LDS and accumulates A~_o * M on the
// MFMA units in registers; the result of each (target, c) is stored by the
// item's first part and added to by later parts.  Complex products use four
// real products: Re += Ar Br - Ai Bi, Im += Ar Bi + Ai Br.  Wave w owns rows
// 32w .. 32w+31 of the (padded) K rows.
//
// This file: bank generation, the work-list kernel and the dispatch to the
// per-precision coupling kernels (m2l_f64.hip, m2l_f32.hip, m2l_bf16.hip).
//
// Items are described by per-(plan, level) descriptors, so one launch can
// serve many plans (a batch); near-field items (one thread per target point)
// can share the launch.  Workgroups either take one item each (grid launch)
// or stay resident and pull items from a device queue (an atomic counter)
// until it is empty (persistent launch).
#include "m2l_device.hpp"

namespace fdm {

namespace {

// Coupling matrices in the layout of the plan precision: FP64 or FP32 split
// re/im planes, k-major (PLANES 2); for the BF16 split precisions, each
// FP32-rounded part split into hi = bf16(x) and lo = bf16(x - hi), four
// planes (PLANES 4), or each FP64 part into hi, mid, lo (see bf16_split3),
// six planes (PLANES 6), in fragment order.  One workgroup per matrix
// (grid-stride over matrices); matrix i of the list is written at position
// i of `bank`.
template <class T, int PLANES>
__global__ void __launch_bounds__(256) k_bank(const int32_t* __restrict__ info,
                                              int64_t n_mat, const BankLevel* __restrict__ lv,
                                              Interp ip, T* __restrict__ bank) {
  const int Kp = ip.Kp, K = ip.K, m1 = ip.m1;
  const int per = Kp * Kp;
  constexpr int planes = PLANES;
  for (int64_t id = blockIdx.x; id < n_mat; id += gridDim.x) {
    const int32_t* in = info + 5 * id;
    const BankLevel L = lv[in[0]];
    const double o[3] = {double(in[1]), double(in[2]), double(in[3])};
    const double* cv = L.dirvec + 3 * in[4];
    const double c0 = cv[0], c1 = cv[1], c2 = cv[2];
    T* base = bank + id * planes * int64_t(per);
    for (int r = threadIdx.x; r < per; r += blockDim.x) {
      const int kk = r / Kp;         // source node (column of A)
      const int row = r - kk * Kp;   // target node (row of A)
      double re = 0.0, im = 0.0;
      if (row < K && kk < K) {
        const int a[3] = {row / (m1 * m1), (row / m1) % m1, row % m1};
        const int b[3] = {kk / (m1 * m1), (kk / m1) % m1, kk % m1};
        double d[3], rel[3];
        for (int q = 0; q < 3; ++q) {
          rel[q] = 0.5 * L.h[q] * (ip.node[a[q]] - ip.node[b[q]]);
          d[q] = L.h[q] * o[q] + rel[q];
        }
        const double rr = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
        const double arg = L.kappa * rr - L.kappa * (rel[0] * c0 + rel[1] * c1 + rel[2] * c2);
        double sn, cs;
        phase_sincos(arg, sn, cs);
        const double w = 1.0 / (4.0 * M_PI * rr);
        re = cs * w;
        im = sn * w;
      }
      if constexpr (PLANES == 6) {
        // six planes (re hi, mid, lo, im hi, mid, lo) in MFMA operand order
        const int f = frag_index(row, kk, Kp);
        uint16_t h, m, l;
        bf16_split3(re, h, m, l);
        base[f] = h;
        base[per + f] = m;
        base[2 * per + f] = l;
        bf16_split3(im, h, m, l);
        base[3 * per + f] = h;
        base[4 * per + f] = m;
        base[5 * per + f] = l;
      } else if constexpr (PLANES == 4) {
        // four planes (re hi, re lo, im hi, im lo) in MFMA operand order
        const int f = frag_index(row, kk, Kp);
        const float fr = static_cast<float>(re), fi = static_cast<float>(im);
        const uint16_t rh = bf16_bits(fr), ih = bf16_bits(fi);
        base[f] = rh;
        base[per + f] = bf16_bits(fr - bf16_value(rh));
        base[2 * per + f] = ih;
        base[3 * per + f] = bf16_bits(fi - bf16_value(ih));
      } else {
        base[kk * Kp + row] = static_cast<T>(re);
        base[per + kk * Kp + row] = static_cast<T>(im);
      }
    }
  }
}


// --------------------------------------------------------- work lists --
// Candidate offsets of an item whose source box is non-empty for at least
// one target of the block: count (pass 0) or write (pass 1) them.  One wave
// per item (<= 64 targets); pass 1 also counts the admissible blocks per
// offset and, per item, the 32-column tiles of the compacted form.
__global__ void __launch_bounds__(64) k_valid_offsets(
    const M2LItem* __restrict__ items, int64_t n_items, const int32_t* __restrict__ cand_begin,
    const int32_t* __restrict__ cand_count, const int32_t* __restrict__ cand,
    const M2LDesc* __restrict__ descs, const int32_t* __restrict__ tgt_list,
    const int4* __restrict__ offtab, int pass, int32_t* __restrict__ counts,
    const int32_t* __restrict__ out_begin, int32_t* __restrict__ out,
    unsigned long long* __restrict__ blocks_per_off, int32_t* __restrict__ tiles) {
  const int lane = threadIdx.x;
  for (int64_t ii = blockIdx.x; ii < n_items; ii += gridDim.x) {
    const M2LItem it = items[ii];
    const M2LDesc D = descs[it.desc];
    const int lim = 1 << D.level;
    int ix = 0, iy = 0, iz = 0;
    const int32_t t = lane < it.ntgt ? tgt_list[it.tgt_begin + lane] : -1;
    if (t >= 0) demorton3(D.keyT[t], D.level, ix, iy, iz);
    const int32_t* cl = cand + cand_begin[ii];
    const int nc = cand_count[ii];
    int n = 0, nt = 0;
    for (int q = 0; q < nc; ++q) {
      const int4 od = offtab[cl[q]];
      bool ok = false;
      if (t >= 0) {
        const int sx = ix - od.x, sy = iy - od.y, sz = iz - od.z;
        if (sx >= 0 && sy >= 0 && sz >= 0 && sx < lim && sy < lim && sz < lim)
          ok = D.gridS[morton3(sx, sy, sz, D.level)] >= 0;
      }
      const unsigned long long mask = __ballot(ok);
      if (mask) {
        if (pass == 1 && lane == 0) {
          out[out_begin[ii] + n] = cl[q];
          atomicAdd(&blocks_per_off[cl[q]], (unsigned long long)__popcll(mask));
        }
        nt += (__popcll(mask) + 31) / 32;
        ++n;
      }
    }
    if (pass == 0 && lane == 0) counts[ii] = n;
    if (pass == 1 && lane == 0) tiles[ii] = nt;
  }
}

}  // namespace

// Row blocks of a coupling matrix of Kp rows, and the workgroup size: one
// wave per 32 rows of a block, at least 8 waves.
int m2l_row_blocks(int Kp) { return (Kp + kMaxKp - 1) / kMaxKp; }

int m2l_threads(int Kp) {
  const int rb = m2l_row_blocks(Kp);
  const int rows = ((Kp + rb - 1) / rb + 31) / 32 * 32;
  return std::max(2 * rows, 512);
}

int64_t m2l_resident_groups(int prec, int nb, int Kp, bool parts) {
  if (prec == FDM_PREC_FP64) return resident_f64(nb, Kp, parts);
  if (prec == FDM_PREC_BF16X3) return resident_bf16(nb, Kp, parts);
  if (prec == FDM_PREC_BF16X6) return resident_bf16x6(nb, Kp, parts);
  return resident_f32(nb, Kp, parts);
}

void launch_m2l_items(const M2LLaunch& L, int prec, int Kp, const TuneConfig& cfg,
                      int32_t* head, hipStream_t s) {
  if (L.n_items == 0) return;
  if (L.n_items > INT32_MAX / 2) fail(FDM_ERR_UNSUPPORTED, "too many coupling items");
  const bool persistent = cfg.persistent && head != nullptr;
  if (L.stage) {
    launch_items_aca(L, L.stage, Kp, persistent, head, s);
    return;
  }
  if (prec == FDM_PREC_FP64)
    launch_items_f64(L, Kp, cfg.nb, persistent, head, s);
  else if (prec == FDM_PREC_BF16X3)
    launch_items_bf16(L, Kp, cfg.nb, persistent, head, s);
  else if (prec == FDM_PREC_BF16X6)
    launch_items_bf16x6(L, Kp, cfg.nb, persistent, head, s);
  else
    launch_items_f32(L, Kp, cfg.nb, persistent, head, s);
}

void launch_bank_direct(const int32_t* info, int64_t n_mat, const BankLevel* lv, int prec,
                        const Interp& ip, void* dst, hipStream_t s) {
  if (n_mat == 0) return;
  const unsigned grid = static_cast<unsigned>(std::min<int64_t>(n_mat, 1 << 16));
  if (prec == FDM_PREC_FP64)
    k_bank<double, 2><<<grid, 256, 0, s>>>(info, n_mat, lv, ip, static_cast<double*>(dst));
  else if (prec == FDM_PREC_BF16X3)
    k_bank<uint16_t, 4><<<grid, 256, 0, s>>>(info, n_mat, lv, ip, static_cast<uint16_t*>(dst));
  else if (prec == FDM_PREC_BF16X6)
    k_bank<uint16_t, 6><<<grid, 256, 0, s>>>(info, n_mat, lv, ip, static_cast<uint16_t*>(dst));
  else
    k_bank<float, 2><<<grid, 256, 0, s>>>(info, n_mat, lv, ip, static_cast<float*>(dst));
  FDM_LAUNCH("k_bank");
}

void launch_bank_matrices(const M2LLaunch& L, int prec, const Interp& ip, hipStream_t s) {
  launch_bank_direct(L.gen_info.get(), L.n_gen, L.gen_levels.get(), prec, ip, L.gen_dst, s);
}

void launch_valid_offsets(const M2LItem* items, int64_t n_items, const int32_t* cand_begin,
                          const int32_t* cand_count, const int32_t* cand, const M2LDesc* descs,
                          const int32_t* tgt_list, const int4* offtab, int pass,
                          int32_t* counts, const int32_t* out_begin, int32_t* out,
                          unsigned long long* blocks_per_off, int32_t* tiles,
                          hipStream_t s) {
  if (n_items == 0) return;
  const unsigned G = static_cast<unsigned>(std::min<int64_t>(n_items, 1 << 16));
  k_valid_offsets<<<G, 64, 0, s>>>(items, n_items, cand_begin, cand_count, cand, descs,
                                   tgt_list, offtab, pass, counts, out_begin, out,
                                   blocks_per_off, tiles);
  FDM_LAUNCH("k_valid_offsets");
}

}  // namespace fdm
