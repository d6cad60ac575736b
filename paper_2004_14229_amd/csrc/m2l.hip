// Coupling step of Alg. 4 (Sect. 2.6, M2L): g~_{t,c} = sum_s A~_{c,t x s} v~_{s,c}
// over the admissible blocks, on the matrix cores.
//
// Bank (Sect. 2.7): the coupling matrix of a block depends only on its level
// and offset o = i_t - i_s, so one K x K complex matrix is stored per
// admissible (level, offset):
//   A~[j,k] = f(xi_{t,j}, xi_{s,k}) exp(-i kappa <(xi_{t,j}-m_t) - (xi_{s,k}-m_s), c>)
// (the paper's f_c with the plane-wave factors of the box centres moved into
// the moments and locals), evaluated in FP64 and stored as split re/im
// planes, transposed (k-major) so that a wave's rows of one k are contiguous.
//
// Product: one workgroup owns a block of up to 64 target boxes of one level,
// one octant (so they share the list of admissible offsets) and one
// direction c.  It loops over that list's offsets that hit at least one
// non-empty source box, gathers the 64 source moment columns t - o (zero for
// missing boxes) through LDS and accumulates A~_o * M on the MFMA units in
// registers; the result of each (target, c) is written once.  Complex
// products use four real products: Re += Ar Br - Ai Bi, Im += Ar Bi + Ai Br.
// Wave w owns rows 32w .. 32w+31 of the (padded) K rows.
#include <algorithm>
#include <numeric>
#include <type_traits>

#include "plan.hpp"
#include "device_math.hpp"

namespace fdm {

namespace {

typedef float f16v __attribute__((ext_vector_type(16)));
typedef double d4v __attribute__((ext_vector_type(4)));

struct BankLevel {
  double h;
  int level;
  int nd;
  const double* dirvec;
};

// BF16 (bfloat16) helpers: round to nearest even of an FP32 value, as the
// raw 16 bits, and the value of such bits.  Finite inputs only.
__device__ __forceinline__ uint16_t bf16_bits(float x) {
  uint32_t u = __float_as_uint(x);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return static_cast<uint16_t>(u >> 16);
}
__device__ __forceinline__ float bf16_value(uint16_t b) {
  return __uint_as_float(static_cast<uint32_t>(b) << 16);
}

// Position of element (row, k) of one BF16 plane: for each k step of 16 and
// block of 32 rows, the 64 lanes' 8-element A operands of
// v_mfma_f32_32x32x16_bf16 (lane = row % 32 + 32 * (k % 16 >= 8)) are
// contiguous, so one wave reads one step of its rows as 1 KiB in a row.
__host__ __device__ __forceinline__ int64_t frag_index(int row, int k, int Kp) {
  const int ks = k / 16, kr = k % 16;
  const int lane = row % 32 + 32 * (kr / 8);
  return ((int64_t(ks) * (Kp / 32) + row / 32) * 64 + lane) * 8 + (kr % 8);
}

// Coupling matrices in the layout of the plan precision: FP64 or FP32 split
// re/im planes, k-major; or, for the BF16 split precision, each FP32-rounded
// part split into hi = bf16(x) and lo = bf16(x - hi), four planes in
// fragment order.
template <class T>
__global__ void k_bank(const int32_t* __restrict__ info,  // per matrix: level, ox, oy, oz, c
                       int64_t n_mat, const BankLevel* __restrict__ lv, double kappa,
                       Interp ip, T* __restrict__ bank) {
  const int Kp = ip.Kp, K = ip.K, m1 = ip.m1;
  const int64_t per = int64_t(Kp) * Kp;
  const int64_t total = n_mat * per;
  for (int64_t e = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; e < total;
       e += int64_t(gridDim.x) * blockDim.x) {
    const int64_t id = e / per;
    const int64_t r = e % per;
    const int kk = static_cast<int>(r / Kp);   // source node (column of A)
    const int row = static_cast<int>(r % Kp);  // target node (row of A)
    double re = 0.0, im = 0.0;
    if (row < K && kk < K) {
      const int32_t* in = info + 5 * id;
      const BankLevel L = lv[in[0]];
      const int o[3] = {in[1], in[2], in[3]};
      const int c = in[4];
      const int a[3] = {row / (m1 * m1), (row / m1) % m1, row % m1};
      const int b[3] = {kk / (m1 * m1), (kk / m1) % m1, kk % m1};
      double d[3], rel[3];
      for (int q = 0; q < 3; ++q) {
        rel[q] = 0.5 * L.h * (ip.node[a[q]] - ip.node[b[q]]);
        d[q] = L.h * o[q] + rel[q];
      }
      const double rr = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
      const double* cv = L.dirvec + 3 * c;
      const double arg = kappa * rr - kappa * (rel[0] * cv[0] + rel[1] * cv[1] + rel[2] * cv[2]);
      double sn, cs;
      phase_sincos(arg, sn, cs);
      const double w = 1.0 / (4.0 * M_PI * rr);
      re = cs * w;
      im = sn * w;
    }
    if constexpr (std::is_same<T, uint16_t>::value) {
      // four planes (re hi, re lo, im hi, im lo) in MFMA operand order
      T* base = bank + id * 4 * per;
      const int64_t f = frag_index(row, kk, Kp);
      const float fr = static_cast<float>(re), fi = static_cast<float>(im);
      const uint16_t rh = bf16_bits(fr), ih = bf16_bits(fi);
      base[f] = rh;
      base[per + f] = bf16_bits(fr - bf16_value(rh));
      base[2 * per + f] = ih;
      base[3 * per + f] = bf16_bits(fi - bf16_value(ih));
    } else {
      T* base = bank + id * 2 * per;
      base[int64_t(kk) * Kp + row] = static_cast<T>(re);
      base[per + int64_t(kk) * Kp + row] = static_cast<T>(im);
    }
  }
}

// Pointers taken from the per-level descriptors are generic; reading them
// through the global address space gives global (not flat) loads, which do
// not count against the LDS wait counter.
template <class T>
__device__ __forceinline__ const __attribute__((address_space(1))) T* gmem(const T* p) {
  return (const __attribute__((address_space(1))) T*)p;
}
typedef float f4n __attribute__((ext_vector_type(4)));
typedef double d2n __attribute__((ext_vector_type(2)));

// 16-byte global load / store through native vector types.
template <class V>
__device__ __forceinline__ V gload16(const void* p) {
  const f4n raw = *gmem(static_cast<const f4n*>(p));
  V v;
  __builtin_memcpy(&v, &raw, 16);
  return v;
}
__device__ __forceinline__ void gstore16(void* p, double2 v) {
  d2n raw;
  __builtin_memcpy(&raw, &v, 16);
  *(__attribute__((address_space(1))) d2n*)(p) = raw;
}

// Shared prologue: the block's target boxes and their integer positions;
// col[b][j] is the first moment element of target j's source column for the
// offset held in buffer b (or -1: empty or outside the grid).
struct TargetTile {
  int32_t t[kNB];
  int32_t x[kNB], y[kNB], z[kNB];
  int64_t col[2][kNB];
};

__device__ __forceinline__ void load_targets(TargetTile& S, const M2LItem& it,
                                             const M2LLevel& L,
                                             const int32_t* __restrict__ tgt_list) {
  for (int j = threadIdx.x; j < kNB; j += blockDim.x) {
    int32_t t = j < it.ntgt ? tgt_list[it.tgt_begin + j] : -1;
    S.t[j] = t;
    int ix = 0, iy = 0, iz = 0;
    if (t >= 0) demorton3(gmem(L.keyT)[t], L.level, ix, iy, iz);
    S.x[j] = ix;
    S.y[j] = iy;
    S.z[j] = iz;
  }
}

__device__ __forceinline__ void source_columns(TargetTile& S, int buf, const M2LLevel& L,
                                               int4 od, int c, int Kp) {
  const int lim = 1 << L.level;
  for (int j = threadIdx.x; j < kNB; j += blockDim.x) {
    int64_t col = -1;
    if (S.t[j] >= 0) {
      const int sx = S.x[j] - od.x, sy = S.y[j] - od.y, sz = S.z[j] - od.z;
      if (sx >= 0 && sy >= 0 && sz >= 0 && sx < lim && sy < lim && sz < lim) {
        const int32_t sb = gmem(L.gridS)[morton3(sx, sy, sz, L.level)];
        if (sb >= 0) col = (int64_t(sb) * L.nd + c) * Kp;
      }
    }
    S.col[buf][j] = col;
  }
}

// Precision traits of the coupling kernel.  Each wave owns 32 rows of the
// (padded) coupling matrix and all kNB target columns of the block.
//  FP32: v_mfma_f32_32x32x2f32, k-step 2, 2 column tiles of 32, k slab 16.
//  FP64: v_mfma_f64_16x16x4f64, k-step 4, 2 row x 4 column tiles of 16, k slab 8.
struct F32Traits {
  using T = float;
  using V16 = float4;  // 16-byte load unit
  static constexpr int KS = 16;
  static constexpr int NACC = 2;  // accumulator tiles per component
  using Acc = f16v;
};
struct F64Traits {
  using T = double;
  using V16 = double2;
  static constexpr int KS = 8;
  static constexpr int NACC = 8;  // 2 row x 4 column tiles
  using Acc = d4v;
};

template <class Tr>
struct M2LShared {
  TargetTile S;
  typename Tr::T B[2][2][Tr::KS][kNB + 1];  // [buffer][re/im][k][column]
};

// Moment columns of one k slab: kNB columns x KS complex values, staged in
// 16-byte pieces, at most one per thread (the workgroup has >= 512 threads).
template <class Tr>
__device__ __forceinline__ typename Tr::V16 load_cols(const TargetTile& S, int colbuf,
                                                      const typename Tr::T* __restrict__ mom,
                                                      int k0) {
  using V = typename Tr::V16;
  constexpr int EPV = sizeof(V) / sizeof(typename Tr::T);
  constexpr int PPC = Tr::KS * 2 / EPV;  // pieces per column
  static_assert(kNB * PPC <= 512, "one staged piece per thread");
  V val{};
  const int e = threadIdx.x;
  if (e < kNB * PPC) {
    const int64_t col = S.col[colbuf][e / PPC];
    if (col >= 0) val = gload16<V>(mom + 2 * (col + k0) + (e % PPC) * EPV);
  }
  return val;
}

template <class Tr>
__device__ __forceinline__ void store_cols(M2LShared<Tr>& sh, int buf, typename Tr::V16 val) {
  using T = typename Tr::T;
  using V = typename Tr::V16;
  constexpr int EPV = sizeof(V) / sizeof(T);
  constexpr int PPC = Tr::KS * 2 / EPV;
  const int e = threadIdx.x;
  if (e < kNB * PPC) {
    const int j = e / PPC, q = e % PPC;
    const T* v = reinterpret_cast<const T*>(&val);
#pragma unroll
    for (int u = 0; u < EPV / 2; ++u) {
      const int k = q * (EPV / 2) + u;
      sh.B[buf][0][k][j] = v[2 * u];
      sh.B[buf][1][k][j] = v[2 * u + 1];
    }
  }
}

// MFMAs of one k slab for one wave: Re += Ar Br - Ai Bi, Im += Ar Bi + Ai Br.
// The coupling matrix is read straight from the bank (k-major: a wave's rows
// of one k are contiguous).
__device__ __forceinline__ void slab_mfma(d4v (&ar)[8], d4v (&ai)[8],
                                          const M2LShared<F64Traits>& sh, int buf,
                                          const double* __restrict__ Ar,
                                          const double* __restrict__ Ai, int k0, int Kp,
                                          int wave, int lane) {
  const int kl = lane / 16, li = lane % 16;
  double a_r[2][2], a_i[2][2];
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int rs = 0; rs < 2; ++rs) {
      const int64_t ka = int64_t(k0 + 4 * t + kl) * Kp + 32 * wave + 16 * rs + li;
      a_r[t][rs] = Ar[ka];
      a_i[t][rs] = Ai[ka];
    }
#pragma unroll
  for (int t = 0; t < 2; ++t) {
    const int kk = 4 * t;
#pragma unroll
    for (int cs = 0; cs < 4; ++cs) {
      const double b_r = sh.B[buf][0][kk + kl][16 * cs + li];
      const double b_i = sh.B[buf][1][kk + kl][16 * cs + li];
#pragma unroll
      for (int rs = 0; rs < 2; ++rs) {
        d4v& cr = ar[rs * 4 + cs];
        d4v& ci = ai[rs * 4 + cs];
        cr = __builtin_amdgcn_mfma_f64_16x16x4f64(a_r[t][rs], b_r, cr, 0, 0, 0);
        cr = __builtin_amdgcn_mfma_f64_16x16x4f64(-a_i[t][rs], b_i, cr, 0, 0, 0);
        ci = __builtin_amdgcn_mfma_f64_16x16x4f64(a_r[t][rs], b_i, ci, 0, 0, 0);
        ci = __builtin_amdgcn_mfma_f64_16x16x4f64(a_i[t][rs], b_r, ci, 0, 0, 0);
      }
    }
  }
}

// Add (or, for the first flush, store) a wave's accumulated totals into the
// FP64 result of its rows and the block's targets.
__device__ __forceinline__ void flush_rows(const f16v (&tr)[2], const f16v (&ti)[2],
                                           const TargetTile& S, double2* out, int nd, int c,
                                           int Kp, int wave, int lane, bool first) {
#pragma unroll
  for (int cs = 0; cs < 2; ++cs) {
    const int32_t t = S.t[32 * cs + (lane % 32)];
    if (t < 0) continue;
    double2* dst = out + (int64_t(t) * nd + c) * Kp;
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      const int r = 32 * wave + 8 * (i / 4) + 4 * (lane / 32) + (i % 4);
      double2 v = make_double2(tr[cs][i], ti[cs][i]);
      if (!first) {
        const double2 o = gload16<double2>(dst + r);
        v.x += o.x;
        v.y += o.y;
      }
      gstore16(dst + r, v);
    }
  }
}

__device__ __forceinline__ void flush_rows(const d4v (&tr)[8], const d4v (&ti)[8],
                                           const TargetTile& S, double2* out, int nd, int c,
                                           int Kp, int wave, int lane, bool first) {
#pragma unroll
  for (int cs = 0; cs < 4; ++cs) {
    const int32_t t = S.t[16 * cs + (lane % 16)];
    if (t < 0) continue;
    double2* dst = out + (int64_t(t) * nd + c) * Kp;
#pragma unroll
    for (int rs = 0; rs < 2; ++rs)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int r = 32 * wave + 16 * rs + lane / 16 + 4 * i;
        double2 v = make_double2(tr[rs * 4 + cs][i], ti[rs * 4 + cs][i]);
        if (!first) {
          const double2 o = gload16<double2>(dst + r);
          v.x += o.x;
          v.y += o.y;
        }
        gstore16(dst + r, v);
      }
  }
}

template <class A>
__device__ __forceinline__ void zero(A& a) {
  for (auto& x : a)
#pragma unroll
    for (int i = 0; i < static_cast<int>(sizeof(x) / sizeof(x[0])); ++i) x[i] = 0;
}

// The FP64 coupling kernel.  One pipeline step = one (offset, k slab): the
// next step's moment columns are loaded into a register before this step's
// MFMAs and stored to the other LDS buffer after them; one barrier ends each
// step.  One FP64 accumulator chain per (row, target).
__global__ void __launch_bounds__(kM2LMaxThreads) k_m2l_f64(
    const M2LItem* __restrict__ items, const M2LLevel* __restrict__ lv,
    const int32_t* __restrict__ tgt_list, const int32_t* __restrict__ valid_off,
    const int4* __restrict__ offtab, const double* __restrict__ bank, int Kp) {
  using Tr = F64Traits;
  __shared__ M2LShared<Tr> sh;
  const M2LItem it = items[blockIdx.x];
  const M2LLevel L = lv[it.level];
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  const bool rows_here = 32 * wave < Kp;  // waves past Kp only help with loads
  load_targets(sh.S, it, L, tgt_list);
  __syncthreads();
  double2* out = static_cast<double2*>(L.out);
  d4v acr[Tr::NACC], aci[Tr::NACC];
  zero(acr);
  zero(aci);
  const int nv = it.vo_count;
  if (nv > 0) {
    const double* mom = static_cast<const double*>(L.mom);
    const int64_t per = int64_t(Kp) * Kp;
    const int ns = Kp / Tr::KS;  // k slabs per offset (>= 2)
    const int total = nv * ns;
    int4 od_cur = offtab[valid_off[it.vo_begin]];
    int4 od_next = od_cur;
    source_columns(sh.S, 0, L, od_cur, it.c, Kp);
    __syncthreads();
    store_cols<Tr>(sh, 0, load_cols<Tr>(sh.S, 0, mom, 0));
    __syncthreads();
    for (int q = 0; q < total; ++q) {
      const int v = q / ns, s = q % ns, cur = q & 1;
      if (s == 0) {
        od_cur = od_next;
        if (v + 1 < nv) {  // source columns of the next offset
          od_next = offtab[valid_off[it.vo_begin + v + 1]];
          source_columns(sh.S, (v + 1) & 1, L, od_next, it.c, Kp);
        }
      }
      const bool more = q + 1 < total;
      double2 nxt{};
      if (more) nxt = load_cols<Tr>(sh.S, ((q + 1) / ns) & 1, mom, ((q + 1) % ns) * Tr::KS);
      if (rows_here) {
        const double* Ar = bank + int64_t(od_cur.w) * 2 * per;
        slab_mfma(acr, aci, sh, cur, Ar, Ar + per, s * Tr::KS, Kp, wave, lane);
      }
      if (more) store_cols<Tr>(sh, cur ^ 1, nxt);
      __syncthreads();
    }
  }
  if (rows_here) flush_rows(acr, aci, sh.S, out, L.nd, it.c, Kp, wave, lane, true);
}

__device__ __forceinline__ void load_a32(float (&a)[2][8], const float* __restrict__ Ar,
                                         int64_t per, int k0, int Kp, int wave, int lane) {
  const int r = 32 * wave + (lane % 32), kl = lane / 32;
#pragma unroll
  for (int t = 0; t < 8; ++t) {
    const int64_t ka = int64_t(k0 + 2 * t + kl) * Kp + r;
    a[0][t] = Ar[ka];
    a[1][t] = Ar[per + ka];
  }
}

__device__ __forceinline__ void mfma32(f16v (&ar)[2], f16v (&ai)[2], const float (&a)[2][8],
                                       const M2LShared<F32Traits>& sh, int buf, int lane) {
  const int kl = lane / 32, cl = lane % 32;
#pragma unroll
  for (int t = 0; t < 8; ++t) {
    const int kk = 2 * t;
#pragma unroll
    for (int cs = 0; cs < 2; ++cs) {
      const float b_r = sh.B[buf][0][kk + kl][32 * cs + cl];
      const float b_i = sh.B[buf][1][kk + kl][32 * cs + cl];
      ar[cs] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[0][t], b_r, ar[cs], 0, 0, 0);
      ar[cs] = __builtin_amdgcn_mfma_f32_32x32x2f32(-a[1][t], b_i, ar[cs], 0, 0, 0);
      ai[cs] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[0][t], b_i, ai[cs], 0, 0, 0);
      ai[cs] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[1][t], b_r, ai[cs], 0, 0, 0);
    }
  }
}

// The FP32 coupling kernel.  Same pipeline.  Each offset's product is summed
// in fresh FP32 accumulators (rounding relative to that product, not to the
// total over all offsets), added to FP32 totals, and every kFlush offsets
// the totals are added to the FP64 result in memory, which this workgroup
// alone owns.
constexpr int kFlush = 16;

__global__ void __launch_bounds__(kM2LMaxThreads) k_m2l_f32(
    const M2LItem* __restrict__ items, const M2LLevel* __restrict__ lv,
    const int32_t* __restrict__ tgt_list, const int32_t* __restrict__ valid_off,
    const int4* __restrict__ offtab, const float* __restrict__ bank, int Kp) {
  using Tr = F32Traits;
  __shared__ M2LShared<Tr> sh;
  const M2LItem it = items[blockIdx.x];
  const M2LLevel L = lv[it.level];
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  const bool rows_here = 32 * wave < Kp;
  load_targets(sh.S, it, L, tgt_list);
  __syncthreads();
  double2* out = static_cast<double2*>(L.out);
  f16v acr[2], aci[2], tor[2], toi[2];
  zero(acr);
  zero(aci);
  const int nv = it.vo_count;
  if (nv == 0) {  // no source box: the result is zero
    if (rows_here) flush_rows(acr, aci, sh.S, out, L.nd, it.c, Kp, wave, lane, true);
    return;
  }
  zero(tor);
  zero(toi);
  const float* mom = static_cast<const float*>(L.mom);
  const int64_t per = int64_t(Kp) * Kp;
  const int ns = Kp / Tr::KS;  // k slabs per offset (>= 2)
  const int total = nv * ns;
  int4 od_cur = offtab[valid_off[it.vo_begin]];
  int4 od_next = od_cur;
  source_columns(sh.S, 0, L, od_cur, it.c, Kp);
  __syncthreads();
  store_cols<Tr>(sh, 0, load_cols<Tr>(sh.S, 0, mom, 0));
  __syncthreads();
  bool first = true;
  for (int q = 0; q < total; ++q) {
    const int v = q / ns, s = q % ns, cur = q & 1;
    if (s == 0) {
      od_cur = od_next;
      if (v + 1 < nv) {  // source columns of the next offset
        od_next = offtab[valid_off[it.vo_begin + v + 1]];
        source_columns(sh.S, (v + 1) & 1, L, od_next, it.c, Kp);
      }
    }
    const bool more = q + 1 < total;
    float4 nxt{};
    if (more) nxt = load_cols<Tr>(sh.S, ((q + 1) / ns) & 1, mom, ((q + 1) % ns) * Tr::KS);
    if (rows_here) {
      if (s == 0) {
        zero(acr);
        zero(aci);
      }
      float a[2][8];
      load_a32(a, bank + int64_t(od_cur.w) * 2 * per, per, s * Tr::KS, Kp, wave, lane);
      mfma32(acr, aci, a, sh, cur, lane);
      if (s == ns - 1) {
#pragma unroll
        for (int c2 = 0; c2 < 2; ++c2) {
          tor[c2] += acr[c2];
          toi[c2] += aci[c2];
        }
        if ((v + 1) % kFlush == 0 || v + 1 == nv) {
          flush_rows(tor, toi, sh.S, out, L.nd, it.c, Kp, wave, lane, first);
          first = false;
          zero(tor);
          zero(toi);
        }
      }
    }
    if (more) store_cols<Tr>(sh, cur ^ 1, nxt);
    __syncthreads();
  }
}

// ------------------------------------------------- BF16 split precision --
// Each real operand x (coupling entry or moment, FP32) is split into two
// BF16 parts x = hi + lo + O(2^-16 |x|), and a real product X Y is taken as
// Xh Yh + Xh Yl + Xl Yh (three v_mfma_f32_32x32x16_bf16, FP32 accumulation);
// the dropped Xl Yl term is of relative size 2^-16.  Complex products as
// above; the FP32 per-offset sums, FP32 totals and FP64 flushes are those of
// the FP32 kernel.
typedef __bf16 bf8v __attribute__((ext_vector_type(8)));
typedef unsigned int u4v __attribute__((ext_vector_type(4)));

struct BF16Shared {
  TargetTile S;
  // [buffer][plane: re hi, re lo, im hi, im lo][column][k]: 16 k per slab,
  // rows padded to 24 (48 bytes) so that 16 lanes' 16-byte reads of 16
  // consecutive columns fall in distinct banks
  alignas(16) uint16_t B[2][4][kNB][24];
};
constexpr int kBKS = 16;  // k per slab

__device__ __forceinline__ void store_cols_bf16(BF16Shared& sh, int buf, float4 val) {
  const int e = threadIdx.x;
  if (e < kNB * 8) {  // piece e: column e / 8, k = 2 (e % 8) and 2 (e % 8) + 1
    const int j = e / 8, k = 2 * (e % 8);
    const uint16_t rh0 = bf16_bits(val.x), ih0 = bf16_bits(val.y);
    const uint16_t rh1 = bf16_bits(val.z), ih1 = bf16_bits(val.w);
    const uint16_t rl0 = bf16_bits(val.x - bf16_value(rh0));
    const uint16_t il0 = bf16_bits(val.y - bf16_value(ih0));
    const uint16_t rl1 = bf16_bits(val.z - bf16_value(rh1));
    const uint16_t il1 = bf16_bits(val.w - bf16_value(ih1));
    auto put = [&](int plane, uint16_t a, uint16_t b) {
      *reinterpret_cast<uint32_t*>(&sh.B[buf][plane][j][k]) =
          uint32_t(a) | (uint32_t(b) << 16);
    };
    put(0, rh0, rh1);
    put(1, rl0, rl1);
    put(2, ih0, ih1);
    put(3, il0, il1);
  }
}

__device__ __forceinline__ bf8v as_bf8(u4v v) {
  bf8v r;
  __builtin_memcpy(&r, &v, 16);
  return r;
}

__device__ __forceinline__ bf8v lds_bf8(const uint16_t* p) {
  return as_bf8(*reinterpret_cast<const u4v*>(p));
}
__device__ __forceinline__ bf8v neg_bf8(bf8v x) {
  const u4v sign = {0x80008000u, 0x80008000u, 0x80008000u, 0x80008000u};
  u4v u;
  __builtin_memcpy(&u, &x, 16);
  return as_bf8(u ^ sign);
}

// One k slab (one MFMA k step) for one wave: A operands from the bank in
// fragment order, B operands from LDS.  Two passes keep few operands live:
// first the A lo parts against the B hi parts, then the A hi parts against
// both B parts.
__device__ __forceinline__ void mfma_bf16x3(f16v (&ar)[2], f16v (&ai)[2],
                                            const uint16_t* __restrict__ A, int64_t per,
                                            const BF16Shared& sh, int buf, int s, int Kp,
                                            int wave, int lane) {
  const int64_t f = ((int64_t(s) * (Kp / 32) + wave) * 64 + lane) * 8;
  const int kq = 8 * (lane / 32);
  {
    const bf8v arl = as_bf8(gload16<u4v>(A + per + f));
    const bf8v ail = as_bf8(gload16<u4v>(A + 3 * per + f));
#pragma unroll
    for (int cs = 0; cs < 2; ++cs) {
      const int col = 32 * cs + lane % 32;
      const bf8v brh = lds_bf8(&sh.B[buf][0][col][kq]);
      const bf8v bih = lds_bf8(&sh.B[buf][2][col][kq]);
      ar[cs] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(arl, brh, ar[cs], 0, 0, 0);
      ai[cs] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(arl, bih, ai[cs], 0, 0, 0);
      ar[cs] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ail, neg_bf8(bih), ar[cs], 0, 0, 0);
      ai[cs] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ail, brh, ai[cs], 0, 0, 0);
      __builtin_amdgcn_sched_barrier(0);
    }
  }
  const bf8v arh = as_bf8(gload16<u4v>(A + f));
  const bf8v aih = as_bf8(gload16<u4v>(A + 2 * per + f));
#pragma unroll
  for (int cs = 0; cs < 2; ++cs) {
    const int col = 32 * cs + lane % 32;
    const bf8v brh = lds_bf8(&sh.B[buf][0][col][kq]);
    const bf8v brl = lds_bf8(&sh.B[buf][1][col][kq]);
    const bf8v bih = lds_bf8(&sh.B[buf][2][col][kq]);
    const bf8v bil = lds_bf8(&sh.B[buf][3][col][kq]);
    f16v r = ar[cs], i = ai[cs];
    r = __builtin_amdgcn_mfma_f32_32x32x16_bf16(arh, brl, r, 0, 0, 0);
    i = __builtin_amdgcn_mfma_f32_32x32x16_bf16(arh, bil, i, 0, 0, 0);
    r = __builtin_amdgcn_mfma_f32_32x32x16_bf16(aih, neg_bf8(bil), r, 0, 0, 0);
    i = __builtin_amdgcn_mfma_f32_32x32x16_bf16(aih, brl, i, 0, 0, 0);
    r = __builtin_amdgcn_mfma_f32_32x32x16_bf16(arh, brh, r, 0, 0, 0);
    i = __builtin_amdgcn_mfma_f32_32x32x16_bf16(arh, bih, i, 0, 0, 0);
    r = __builtin_amdgcn_mfma_f32_32x32x16_bf16(aih, neg_bf8(bih), r, 0, 0, 0);
    i = __builtin_amdgcn_mfma_f32_32x32x16_bf16(aih, brh, i, 0, 0, 0);
    ar[cs] = r;
    ai[cs] = i;
    __builtin_amdgcn_sched_barrier(0);
  }
}

__global__ void __launch_bounds__(kM2LMaxThreads) k_m2l_bf16x3(
    const M2LItem* __restrict__ items, const M2LLevel* __restrict__ lv,
    const int32_t* __restrict__ tgt_list, const int32_t* __restrict__ valid_off,
    const int4* __restrict__ offtab, const uint16_t* __restrict__ bank, int Kp) {
  __shared__ BF16Shared sh;
  const M2LItem it = items[blockIdx.x];
  const M2LLevel L = lv[it.level];
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  const bool rows_here = 32 * wave < Kp;
  load_targets(sh.S, it, L, tgt_list);
  __syncthreads();
  double2* out = static_cast<double2*>(L.out);
  f16v acr[2], aci[2], tor[2], toi[2];
  zero(acr);
  zero(aci);
  const int nv = it.vo_count;
  if (nv == 0) {  // no source box: the result is zero
    if (rows_here) flush_rows(acr, aci, sh.S, out, L.nd, it.c, Kp, wave, lane, true);
    return;
  }
  zero(tor);
  zero(toi);
  const float* mom = static_cast<const float*>(L.mom);
  const int64_t per = int64_t(Kp) * Kp;
  const int ns = Kp / kBKS;  // k slabs per offset
  const int total = nv * ns;
  int4 od_cur = offtab[valid_off[it.vo_begin]];
  int4 od_next = od_cur;
  source_columns(sh.S, 0, L, od_cur, it.c, Kp);
  __syncthreads();
  store_cols_bf16(sh, 0, load_cols<F32Traits>(sh.S, 0, mom, 0));
  __syncthreads();
  bool first = true;
  for (int q = 0; q < total; ++q) {
    const int v = q / ns, s = q % ns, cur = q & 1;
    if (s == 0) {
      od_cur = od_next;
      if (v + 1 < nv) {  // source columns of the next offset
        od_next = offtab[valid_off[it.vo_begin + v + 1]];
        source_columns(sh.S, (v + 1) & 1, L, od_next, it.c, Kp);
      }
    }
    const bool more = q + 1 < total;
    float4 nxt{};
    if (more)
      nxt = load_cols<F32Traits>(sh.S, ((q + 1) / ns) & 1, mom, ((q + 1) % ns) * kBKS);
    if (rows_here) {
      if (s == 0) {
        zero(acr);
        zero(aci);
      }
      mfma_bf16x3(acr, aci, bank + int64_t(od_cur.w) * 4 * per, per, sh, cur, s, Kp, wave,
                  lane);
      if (s == ns - 1) {
#pragma unroll
        for (int c2 = 0; c2 < 2; ++c2) {
          tor[c2] += acr[c2];
          toi[c2] += aci[c2];
        }
        if ((v + 1) % kFlush == 0 || v + 1 == nv) {
          flush_rows(tor, toi, sh.S, out, L.nd, it.c, Kp, wave, lane, first);
          first = false;
          zero(tor);
          zero(toi);
        }
      }
    }
    if (more) store_cols_bf16(sh, cur ^ 1, nxt);
    __syncthreads();
  }
}

// --------------------------------------------------------- work lists --
// Candidate offsets of an item whose source box is non-empty for at least
// one target of the block: count (pass 0) or write (pass 1) them.  One wave
// per item; also counts the admissible blocks per offset.
__global__ void __launch_bounds__(64) k_valid_offsets(
    const M2LItem* __restrict__ items, int64_t n_items, const int32_t* __restrict__ cand_begin,
    const int32_t* __restrict__ cand_count, const int32_t* __restrict__ cand,
    const M2LLevel* __restrict__ lv, const int32_t* __restrict__ tgt_list,
    const int4* __restrict__ offtab, int pass, int32_t* __restrict__ counts,
    const int32_t* __restrict__ out_begin, int32_t* __restrict__ out,
    unsigned long long* __restrict__ blocks_per_off) {
  const int lane = threadIdx.x;
  for (int64_t ii = blockIdx.x; ii < n_items; ii += gridDim.x) {
    const M2LItem it = items[ii];
    const M2LLevel L = lv[it.level];
    const int lim = 1 << L.level;
    int ix = 0, iy = 0, iz = 0;
    const int32_t t = lane < it.ntgt ? tgt_list[it.tgt_begin + lane] : -1;
    if (t >= 0) demorton3(L.keyT[t], L.level, ix, iy, iz);
    const int32_t* cl = cand + cand_begin[ii];
    const int nc = cand_count[ii];
    int n = 0;
    for (int q = 0; q < nc; ++q) {
      const int4 od = offtab[cl[q]];
      bool ok = false;
      if (t >= 0) {
        const int sx = ix - od.x, sy = iy - od.y, sz = iz - od.z;
        if (sx >= 0 && sy >= 0 && sz >= 0 && sx < lim && sy < lim && sz < lim)
          ok = L.gridS[morton3(sx, sy, sz, L.level)] >= 0;
      }
      const unsigned long long mask = __ballot(ok);
      if (mask) {
        if (pass == 1 && lane == 0) {
          out[out_begin[ii] + n] = cl[q];
          atomicAdd(&blocks_per_off[cl[q]], (unsigned long long)__popcll(mask));
        }
        ++n;
      }
    }
    if (pass == 0 && lane == 0) counts[ii] = n;
  }
}

}  // namespace

void launch_bank(Plan& P, hipStream_t s) {
  if (P.n_bank == 0) return;
  std::vector<int32_t> info;
  info.reserve(5 * P.n_bank);
  std::vector<BankLevel> bl(P.levels + 1);
  for (int l = 0; l <= P.levels; ++l) {
    bl[l] = BankLevel{P.L[l].h, l, P.L[l].nd, P.L[l].dirvec.get()};
    const LevelTable& T = P.tab[l];
    for (size_t i = 0; i < T.adm.size(); ++i) {
      info.push_back(l);
      info.push_back(T.adm[i].x);
      info.push_back(T.adm[i].y);
      info.push_back(T.adm[i].z);
      info.push_back(T.dir[i]);
    }
  }
  DevBuf<int32_t> d_info;
  DevBuf<BankLevel> d_bl;
  to_device(d_info, info, s, nullptr);
  to_device(d_bl, bl, s, nullptr);
  const int64_t per = int64_t(P.ip.Kp) * P.ip.Kp;
  const int64_t total = P.n_bank * per;
  const int B = 256;
  if (P.prec == FDM_PREC_FP64) {
    P.bank64.alloc(2 * total, &P.tally);
    k_bank<double><<<grid_for(total, B), B, 0, s>>>(d_info.get(), P.n_bank, d_bl.get(),
                                                  P.kappa, P.ip, P.bank64.get());
  } else if (P.prec == FDM_PREC_BF16X3) {
    P.bank16.alloc(4 * total, &P.tally);
    k_bank<uint16_t><<<grid_for(total, B), B, 0, s>>>(d_info.get(), P.n_bank, d_bl.get(),
                                                    P.kappa, P.ip, P.bank16.get());
  } else {
    P.bank32.alloc(2 * total, &P.tally);
    k_bank<float><<<grid_for(total, B), B, 0, s>>>(d_info.get(), P.n_bank, d_bl.get(),
                                                 P.kappa, P.ip, P.bank32.get());
  }
  FDM_LAUNCH("k_bank");
  FDM_HIP(hipStreamSynchronize(s));
}

void build_m2l_work(Plan& P, hipStream_t s) {
  const int p = P.levels;
  std::vector<M2LItem> items;
  std::vector<int32_t> tgt_list, cand, cand_begin_per_item, cand_count_per_item;
  std::vector<int4> offtab(P.n_bank);
  std::vector<M2LLevel> lv(p + 1);
  for (int l = 0; l <= p; ++l) {
    const LevelTable& T = P.tab[l];
    LevelData& Ld = P.L[l];
    for (size_t i = 0; i < T.adm.size(); ++i)
      offtab[Ld.bank_base + i] = make_int4(T.adm[i].x, T.adm[i].y, T.adm[i].z,
                                           static_cast<int>(Ld.bank_base + i));
    M2LLevel m{};
    m.gridS = P.S.grid[l].get();
    m.keyT = P.T.key[l].get();
    m.nd = Ld.nd;
    m.level = l;
    m.mom = P.prec == FDM_PREC_FP64 ? static_cast<const void*>(Ld.mom64.get())
                                    : static_cast<const void*>(Ld.mom32.get());
    m.out = Ld.loc64.get();  // FP64 coupling result, completed in place by L2L
    lv[l] = m;
  }
  for (int l = std::max(P.l_min, 0); l <= p; ++l) {
    const LevelTable& T = P.tab[l];
    const LevelData& Ld = P.L[l];
    // candidate offsets per (octant, direction)
    std::vector<std::vector<int32_t>> lists(8 * Ld.nd);
    for (size_t i = 0; i < T.adm.size(); ++i)
      for (int q = 0; q < 8; ++q)
        if (T.mask[i] & (1u << q))
          lists[q * Ld.nd + T.dir[i]].push_back(static_cast<int32_t>(Ld.bank_base + i));
    std::vector<int32_t> list_begin(8 * Ld.nd);
    for (size_t k = 0; k < lists.size(); ++k) {
      list_begin[k] = static_cast<int32_t>(cand.size());
      cand.insert(cand.end(), lists[k].begin(), lists[k].end());
    }
    // target boxes grouped by octant, in Morton order
    std::vector<uint32_t> keys = to_host(P.T.key[l].get(), P.T.nb[l], s);
    std::vector<std::vector<int32_t>> by_oct(8);
    for (size_t b = 0; b < keys.size(); ++b) by_oct[keys[b] & 7].push_back(static_cast<int32_t>(b));
    // items ordered (octant, direction, block): one group per (octant,
    // direction), blocks in Morton order within a group
    for (int q = 0; q < 8; ++q) {
      const auto& bx = by_oct[q];
      std::vector<std::pair<int32_t, int32_t>> blocks;  // (tgt_begin, ntgt)
      for (size_t b0 = 0; b0 < bx.size(); b0 += kNB) {
        const int nt = static_cast<int>(std::min<size_t>(kNB, bx.size() - b0));
        blocks.push_back({static_cast<int32_t>(tgt_list.size()), nt});
        tgt_list.insert(tgt_list.end(), bx.begin() + b0, bx.begin() + b0 + nt);
      }
      for (int c = 0; c < Ld.nd; ++c)
        for (auto [tb, nt] : blocks) {
          items.push_back(M2LItem{l, c, tb, nt, 0, 0});
          cand_begin_per_item.push_back(list_begin[q * Ld.nd + c]);
          cand_count_per_item.push_back(static_cast<int32_t>(lists[q * Ld.nd + c].size()));
        }
    }
  }
  P.n_items = static_cast<int64_t>(items.size());
  to_device(P.m2l_levels, lv, s, &P.tally);
  P.offtab.alloc(P.n_bank, &P.tally);
  if (P.n_bank)
    FDM_HIP(hipMemcpyAsync(P.offtab.get(), offtab.data(), offtab.size() * sizeof(int4),
                           hipMemcpyHostToDevice, s));
  to_device(P.tgt_list, tgt_list, s, &P.tally);
  if (P.n_items == 0) {
    FDM_HIP(hipStreamSynchronize(s));
    return;
  }
  DevBuf<M2LItem> d_items;
  DevBuf<int32_t> d_cand, d_cb, d_cc, d_counts(P.n_items), d_begin;
  to_device(d_items, items, s, nullptr);
  to_device(d_cand, cand, s, nullptr);
  to_device(d_cb, cand_begin_per_item, s, nullptr);
  to_device(d_cc, cand_count_per_item, s, nullptr);
  DevBuf<unsigned long long> d_bpo(std::max<int64_t>(P.n_bank, 1));
  FDM_HIP(hipMemsetAsync(d_bpo.get(), 0, d_bpo.bytes(), s));
  const unsigned G = static_cast<unsigned>(std::min<int64_t>(P.n_items, 1 << 16));
  k_valid_offsets<<<G, 64, 0, s>>>(d_items.get(), P.n_items, d_cb.get(), d_cc.get(),
                                   d_cand.get(), P.m2l_levels.get(), P.tgt_list.get(),
                                   P.offtab.get(), 0, d_counts.get(), nullptr, nullptr,
                                   nullptr);
  FDM_LAUNCH("k_valid_offsets");
  std::vector<int32_t> counts = to_host(d_counts.get(), P.n_items, s);
  std::vector<int32_t> begin(P.n_items);
  int64_t total = 0;
  for (int64_t i = 0; i < P.n_items; ++i) {
    begin[i] = static_cast<int32_t>(total);
    total += counts[i];
  }
  to_device(d_begin, begin, s, nullptr);
  P.valid_off.alloc(std::max<int64_t>(total, 1), &P.tally);
  k_valid_offsets<<<G, 64, 0, s>>>(d_items.get(), P.n_items, d_cb.get(), d_cc.get(),
                                   d_cand.get(), P.m2l_levels.get(), P.tgt_list.get(),
                                   P.offtab.get(), 1, nullptr, d_begin.get(),
                                   P.valid_off.get(), d_bpo.get());
  FDM_LAUNCH("k_valid_offsets");
  std::vector<unsigned long long> bpo = to_host(d_bpo.get(), P.n_bank, s);
  // finish the items: offset ranges
  for (int64_t i = 0; i < P.n_items; ++i) {
    items[i].vo_begin = begin[i];
    items[i].vo_count = counts[i];
  }
  // heaviest items first (longest-processing-time order): measured faster
  // than keeping items of one offset group together on one XCD
  std::stable_sort(items.begin(), items.end(), [](const M2LItem& a, const M2LItem& b) {
    return a.vo_count > b.vo_count;
  });
  to_device(P.items, items, s, &P.tally);
  // statistics and per-level offset use for export
  P.n_couplings = 0;
  P.n_stored = 0;
  P.m2l_columns = total * kNB;
  P.off_used.assign(p + 1, {});
  for (int l = 0; l <= p; ++l) {
    const LevelTable& T = P.tab[l];
    for (size_t i = 0; i < T.adm.size(); ++i) {
      const unsigned long long n = bpo[P.L[l].bank_base + i];
      if (!n) continue;
      P.n_couplings += static_cast<int64_t>(n);
      P.n_stored += 1;
      auto& u = P.off_used[l];
      u.push_back(T.adm[i].x);
      u.push_back(T.adm[i].y);
      u.push_back(T.adm[i].z);
      u.push_back(static_cast<int64_t>(n));
      u.push_back(T.dir[i]);
    }
  }
  FDM_HIP(hipStreamSynchronize(s));
}

void launch_m2l(Plan& P, hipStream_t s) {
  if (P.n_items == 0) return;
  const int threads = std::max(2 * P.ip.Kp, 512);  // one wave per 32 rows, >= 8 waves
  if (P.prec == FDM_PREC_FP64) {
    k_m2l_f64<<<static_cast<unsigned>(P.n_items), threads, 0, s>>>(
        P.items.get(), P.m2l_levels.get(), P.tgt_list.get(), P.valid_off.get(),
        P.offtab.get(), P.bank64.get(), P.ip.Kp);
    FDM_LAUNCH("k_m2l_f64");
  } else if (P.prec == FDM_PREC_BF16X3) {
    k_m2l_bf16x3<<<static_cast<unsigned>(P.n_items), threads, 0, s>>>(
        P.items.get(), P.m2l_levels.get(), P.tgt_list.get(), P.valid_off.get(),
        P.offtab.get(), P.bank16.get(), P.ip.Kp);
    FDM_LAUNCH("k_m2l_bf16x3");
  } else {
    k_m2l_f32<<<static_cast<unsigned>(P.n_items), threads, 0, s>>>(
        P.items.get(), P.m2l_levels.get(), P.tgt_list.get(), P.valid_off.get(),
        P.offtab.get(), P.bank32.get(), P.ip.Kp);
    FDM_LAUNCH("k_m2l_f32");
  }
}

}  // namespace fdm
