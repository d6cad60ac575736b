// Forward transformation of Alg. 4 (Sect. 2.6): S2M on the leaves and M2M
// up to the coarsest level that holds a coupling, in the centre-relative
// phase form:
//
//   S2M  v~_{s,c}[mu] = sum_{k in s} L_{s,mu}(y_k) exp(-i kappa <y_k - m_s, c>) v_k
//   M2M  v~_{s,c} = sum_{s'} E_{s'}^T ( conj(E~d_{s',c}) .* v~_{s',c'} )
//        E~d_{s',c}[k] = exp(i kappa (<xi_{s',k} - m_s, c> - <xi_{s',k} - m_{s'}, c'>))
//
// These equal the paper's moments times exp(i kappa <m_s, c>) (the factor
// moves into the coupling matrices), which keeps every phase argument of
// the size of a box.  E_{s'} (Sect. 2.7) is the tensor product of two 1D
// Lagrange interpolation matrices (child lower / upper half per axis), so it
// is applied as three 1D passes; E~d factorises per axis as well.
// Every direction of D^(l) is formed for every box (a superset of
// D(s) u D^(s); the extra moments are never read).
#include "plan.hpp"
#include "device_math.hpp"

namespace fdm {

namespace {

// Three-part BF16 split of an FP64 value (hi = bf16(fp32(x)), then the same
// of the remainders), as raw bits.
__device__ __forceinline__ void split3_bits(double x, uint16_t& h, uint16_t& m, uint16_t& l) {
  auto bits = [](float f) {
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return static_cast<uint16_t>(u >> 16);
  };
  auto value = [](uint16_t b) { return double(__uint_as_float(uint32_t(b) << 16)); };
  h = bits(static_cast<float>(x));
  const double r1 = x - value(h);
  m = bits(static_cast<float>(r1));
  l = bits(static_cast<float>(r1 - value(m)));
}

// Write one coefficient vector (K values, zero padding up to Kp) in FP64 and,
// if requested, as the FP32 operand copy or as the split BF16 operand copy
// (per slab of 16 coefficients, six planes of 16: re hi, mid, lo, im hi,
// mid, lo); thread `lane` of T holds coefficients lane + T i.
template <int T, int NPER, bool X6 = true>  // X6: out16 may be set
__device__ __forceinline__ void store_coeffs(const double2 (&acc)[NPER],
                                             double2* __restrict__ out64,
                                             float2* __restrict__ out32,
                                             uint16_t* __restrict__ out16,
                                             int64_t base, int K, int Kp, int lane) {
#pragma unroll
  for (int i = 0; i < (kMaxK + T - 1) / T + 1; ++i) {
    const int k = lane + T * i;
    if (k < Kp) {
      const double2 val = (k < K && i < NPER) ? acc[i < NPER ? i : 0]
                                              : make_double2(0.0, 0.0);
      out64[base + k] = val;
      if (out32) out32[base + k] = make_float2(float(val.x), float(val.y));
      if (X6 && out16) {
        uint16_t* d = out16 + 6 * base + 96 * (k / 16) + k % 16;
        uint16_t h, m, l;
        split3_bits(val.x, h, m, l);
        d[0] = h;
        d[16] = m;
        d[32] = l;
        split3_bits(val.y, h, m, l);
        d[48] = h;
        d[64] = m;
        d[80] = l;
      }
    }
  }
}

__global__ void k_permute_in(const double2* __restrict__ v_user,
                             const int32_t* __restrict__ perm, int64_t n,
                             double2* __restrict__ v_tree) {
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * blockDim.x)
    v_tree[i] = v_user[perm[i]];
}

__global__ void k_permute_out(const double2* __restrict__ y_tree,
                              const int32_t* __restrict__ perm, int64_t n,
                              double2* __restrict__ y_user) {
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * blockDim.x)
    y_user[perm[i]] = y_tree[i];
}

__global__ void k_permute_in_c64(const float2* __restrict__ v_user,
                                 const int32_t* __restrict__ perm, int64_t n,
                                 double2* __restrict__ v_tree) {
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * blockDim.x) {
    const float2 a = v_user[perm[i]];
    v_tree[i] = make_double2(a.x, a.y);
  }
}

__global__ void k_permute_out_c64(const double2* __restrict__ y_tree,
                                  const int32_t* __restrict__ perm, int64_t n,
                                  float2* __restrict__ y_user) {
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * blockDim.x)
    y_user[perm[i]] = make_float2(float(y_tree[i].x), float(y_tree[i].y));
}

// One wave per (leaf box, direction); boxes: the listed boxes of the level
// (adaptive trees), or NULL for boxes 0 .. nb-1.  X6: the plan keeps the
// split BF16 moment copy (mom16), else mom16 is NULL and its code is left
// out (fewer registers, more waves in flight for the stores).
// NPER: coefficients per lane, ceil(K / 64) (registers scale with it).
template <bool X6, int NPER>
__global__ void __launch_bounds__(64) k_s2m(
    const double* __restrict__ x, const double* __restrict__ y,
    const double* __restrict__ z, const double2* __restrict__ v,
    const uint32_t* __restrict__ key, const int32_t* __restrict__ start,
    const int32_t* __restrict__ count, const int32_t* __restrict__ boxes, int64_t nb,
    int level, double lo0,
    double lo1, double lo2, double3 h, const double* __restrict__ dirvec, int nd,
    double kappa, Interp ip, double2* __restrict__ mom, float2* __restrict__ mom32,
    uint16_t* __restrict__ mom16) {
  __shared__ double lag[3][kMaxM1];
  const int lane = threadIdx.x;
  const int c = blockIdx.y;
  const int m1 = ip.m1, K = ip.K, Kp = ip.Kp;
  const double cx = dirvec[3 * c], cy = dirvec[3 * c + 1], cz = dirvec[3 * c + 2];
  for (int64_t bi = blockIdx.x; bi < nb; bi += gridDim.x) {
    const int64_t b = boxes ? boxes[bi] : bi;
    int ix, iy, iz;
    demorton3(key[b], level, ix, iy, iz);
    const double mx = lo0 + (ix + 0.5) * h.x, my = lo1 + (iy + 0.5) * h.y,
                 mz = lo2 + (iz + 0.5) * h.z;
    const double inv_half[3] = {2.0 / h.x, 2.0 / h.y, 2.0 / h.z};
    double2 acc[NPER];
    for (int i = 0; i < NPER; ++i) acc[i] = make_double2(0.0, 0.0);
    const int p0 = start[b], pn = count[b];
    for (int pi = 0; pi < pn; ++pi) {
      const int64_t j = p0 + pi;
      const double dx = x[j] - mx, dy = y[j] - my, dz = z[j] - mz;
      __syncthreads();
      if (lane < 3 * m1) {
        const int d = lane / m1, nu = lane % m1;
        const double u = (d == 0 ? dx : d == 1 ? dy : dz) * inv_half[d];
        lag[d][nu] = lagrange1d(ip, nu, u);
      }
      __syncthreads();
      double sn, cs;
      phase_sincos(-kappa * (dx * cx + dy * cy + dz * cz), sn, cs);
      const double2 vj = v[j];
      const double wr = vj.x * cs - vj.y * sn, wi = vj.x * sn + vj.y * cs;
#pragma unroll
      for (int i = 0; i < NPER; ++i) {
        const int mu = lane + 64 * i;
        if (mu < K) {
          const int n3 = mu % m1, n2 = (mu / m1) % m1, n1 = mu / (m1 * m1);
          const double L = lag[0][n1] * lag[1][n2] * lag[2][n3];
          acc[i].x += L * wr;
          acc[i].y += L * wi;
        }
      }
    }
    store_coeffs<64, NPER, X6>(acc, mom, mom32, mom16, (b * nd + c) * int64_t(Kp), K, Kp,
                                   lane);
  }
}

// One workgroup (kXT threads) per (parent box, direction); the children in
// turn, each transformed by the whole workgroup.
__global__ void __launch_bounds__(kXT) k_m2m(
    const double2* __restrict__ child_mom, int nd1, const int32_t* __restrict__ grid1,
    const uint32_t* __restrict__ key, int64_t nb, int level, double3 h1,
    const double* __restrict__ dirvec, const double* __restrict__ dirvec1, int nd,
    int l_hf, double kappa, Interp ip, double2* __restrict__ mom,
    float2* __restrict__ mom32, uint16_t* __restrict__ mom16) {
  __shared__ double2 buf[2][kMaxK];
  __shared__ double2 ph[3][kMaxM1];
  const int lane = threadIdx.x;
  const int c = blockIdx.y;
  const int m1 = ip.m1, K = ip.K, Kp = ip.Kp;
  const int cp = (level + 1 <= l_hf) ? (c >> 2) : 0;  // c' = dir_(l+1)(c)
  const double cv[3] = {dirvec[3 * c], dirvec[3 * c + 1], dirvec[3 * c + 2]};
  const double cv1[3] = {dirvec1[3 * cp], dirvec1[3 * cp + 1], dirvec1[3 * cp + 2]};
  for (int64_t b = blockIdx.x; b < nb; b += gridDim.x) {
    double2 acc[kPerXT];
    for (int i = 0; i < kPerXT; ++i) acc[i] = make_double2(0.0, 0.0);
    const uint32_t pkey = key[b];
    for (int q = 0; q < 8; ++q) {
      const int32_t ch = grid1[(pkey << 3) | q];
      if (ch < 0) continue;
      const int bq[3] = {(q >> 2) & 1, (q >> 1) & 1, q & 1};
      __syncthreads();
      // per-axis factors of conj(E~d): exp(-i kappa ((xi-m_s) c - (xi-m_s') c'))
      if (lane < 3 * m1) {
        const int d = lane / m1, nu = lane % m1;
        const double hd = d == 0 ? h1.x : d == 1 ? h1.y : h1.z;
        const double r = 0.5 * hd * ip.node[nu];          // xi - m_{s'}
        const double off = (bq[d] - 0.5) * hd;            // m_{s'} - m_s
        double sn, cs;
        phase_sincos(-kappa * ((r + off) * cv[d] - r * cv1[d]), sn, cs);
        ph[d][nu] = make_double2(cs, sn);
      }
      __syncthreads();
      const double2* src = child_mom + (int64_t(ch) * nd1 + cp) * Kp;
      for (int k = lane; k < K; k += kXT) {
        const int n3 = k % m1, n2 = (k / m1) % m1, n1 = k / (m1 * m1);
        double2 f = cmul(cmul(ph[0][n1], ph[1][n2]), ph[2][n3]);
        buf[0][k] = cmul(f, src[k]);
      }
      __syncthreads();
      // E_{s'}^T as three 1D passes: out[k] = sum_j E1[b][j][k] in[j]
      apply_transfer(buf, ip, bq, true, lane, kXT);  // result in buf[1]
#pragma unroll
      for (int i = 0; i < kPerXT; ++i) {
        const int k = lane + kXT * i;
        if (k < K) {
          acc[i].x += buf[1][k].x;
          acc[i].y += buf[1][k].y;
        }
      }
    }
    store_coeffs<kXT>(acc, mom, mom32, mom16, (b * nd + c) * int64_t(Kp), K, Kp, lane);
  }
}

// One workgroup (kXT threads) per (parent box, direction), the eight
// children together.  E_{s'}^T is a product of three 1D passes of which
// only the z pass depends on the child's z bit, so for each x half bx the z
// pass takes the four children (by, bz) straight to two sums over bz, the
// y pass those to one sum over by, and the x pass adds it to the result:
// 14 one-dimensional passes per parent instead of 24, and 8 barriers
// instead of 40.  The per-axis phase factors depend only on the child's
// octant bit along that axis, so they are formed once per workgroup.
// Dynamic LDS: 6 K complex values.
__global__ void __launch_bounds__(kXT) k_m2m_oct(
    const double2* __restrict__ child_mom, int nd1, const int32_t* __restrict__ grid1,
    const uint32_t* __restrict__ key, int64_t nb, int level, double3 h1,
    const double* __restrict__ dirvec, const double* __restrict__ dirvec1, int nd,
    int l_hf, double kappa, Interp ip, double2* __restrict__ mom,
    float2* __restrict__ mom32, uint16_t* __restrict__ mom16) {
  extern __shared__ double2 smem[];
  __shared__ double2 ph[3][2][kMaxM1];      // axis, octant bit, node
  __shared__ double e1[2][kMaxM1][kMaxM1];  // E1[b][k][j]
  __shared__ int32_t chs[8];
  const int lane = threadIdx.x;
  const int c = blockIdx.y;
  const int m1 = ip.m1, m2 = m1 * m1, K = ip.K, Kp = ip.Kp;
  double2* in = smem;           // [4][K]: the half's children (by, bz), phased
  double2* mid = smem + 4 * K;  // [2][K]: z pass, summed over bz
  double2* yx = smem;           // [K]: y pass, summed over by (in is read by then)
  const int cp = (level + 1 <= l_hf) ? (c >> 2) : 0;  // c' = dir_(l+1)(c)
  if (lane < 6 * m1) {  // conj(E~d) per axis: exp(-i kappa ((xi-m_s) c - (xi-m_s') c'))
    const int d = lane / (2 * m1), b = (lane / m1) % 2, nu = lane % m1;
    const double hd = d == 0 ? h1.x : d == 1 ? h1.y : h1.z;
    const double r = 0.5 * hd * ip.node[nu];  // xi - m_{s'}
    const double off = (b - 0.5) * hd;        // m_{s'} - m_s
    double sn, cs;
    phase_sincos(-kappa * ((r + off) * dirvec[3 * c + d] - r * dirvec1[3 * cp + d]), sn, cs);
    ph[d][b][nu] = make_double2(cs, sn);
  }
  for (int e = lane; e < 2 * m2; e += kXT) {
    const int b = e / m2, k = (e / m1) % m1, j = e % m1;
    e1[b][k][j] = ip.E1[b][k][j];
  }
  for (int64_t b = blockIdx.x; b < nb; b += gridDim.x) {
    __syncthreads();  // (tables; the previous box's reads of chs)
    if (lane < 8) chs[lane] = grid1[(key[b] << 3) | lane];
    __syncthreads();
    double2 acc[kPerXT];
    for (int i = 0; i < kPerXT; ++i) acc[i] = make_double2(0.0, 0.0);
    for (int bx = 0; bx < 2; ++bx) {
      if (max(max(chs[4 * bx], chs[4 * bx + 1]), max(chs[4 * bx + 2], chs[4 * bx + 3])) < 0)
        continue;  // no child in this half (the same for the whole workgroup)
      for (int e = lane; e < 4 * K; e += kXT) {
        const int i = e / K, k = e - i * K;  // i = 2 by + bz
        const int32_t ch = chs[4 * bx + i];
        double2 v = make_double2(0.0, 0.0);
        if (ch >= 0) {
          const int n1 = k / m2, n2 = (k / m1) % m1, n3 = k % m1;
          const double2 f = cmul(cmul(ph[0][bx][n1], ph[1][i >> 1][n2]), ph[2][i & 1][n3]);
          v = cmul(f, child_mom[(int64_t(ch) * nd1 + cp) * Kp + k]);
        }
        in[e] = v;
      }
      __syncthreads();
      for (int e = lane; e < 2 * K; e += kXT) {  // z pass (stride 1)
        const int by = e / K, ee = e - by * K;
        const int j = ee % m1, base = ee - j;
        double re = 0.0, im = 0.0;
        for (int bz = 0; bz < 2; ++bz) {
          const double2* src = in + (2 * by + bz) * K + base;
          for (int k = 0; k < m1; ++k) {
            const double w = e1[bz][k][j];
            re += w * src[k].x;
            im += w * src[k].y;
          }
        }
        mid[e] = make_double2(re, im);
      }
      __syncthreads();
      for (int e = lane; e < K; e += kXT) {  // y pass (stride m1)
        const int j = (e / m1) % m1, base = e - j * m1;
        double re = 0.0, im = 0.0;
        for (int by = 0; by < 2; ++by) {
          const double2* src = mid + by * K + base;
          for (int k = 0; k < m1; ++k) {
            const double w = e1[by][k][j];
            re += w * src[k * m1].x;
            im += w * src[k * m1].y;
          }
        }
        yx[e] = make_double2(re, im);
      }
      __syncthreads();
#pragma unroll
      for (int i = 0; i < kPerXT; ++i) {  // x pass (stride m1^2) into the result
        const int e = lane + kXT * i;
        if (e < K) {
          const int j = e / m2, base = e - j * m2;
          double re = 0.0, im = 0.0;
          for (int k = 0; k < m1; ++k) {
            const double w = e1[bx][k][j];
            re += w * yx[base + k * m2].x;
            im += w * yx[base + k * m2].y;
          }
          acc[i].x += re;
          acc[i].y += im;
        }
      }
      __syncthreads();  // (yx and in are overwritten by the next half)
    }
    store_coeffs<kXT>(acc, mom, mom32, mom16, (b * nd + c) * int64_t(Kp), K, Kp, lane);
  }
}

}  // namespace

void launch_permute_in(const double* v_user, const int32_t* perm, int64_t n,
                       double* v_tree, hipStream_t s) {
  if (n == 0) return;
  k_permute_in<<<grid_for(n, 256), 256, 0, s>>>(
      reinterpret_cast<const double2*>(v_user), perm, n, reinterpret_cast<double2*>(v_tree));
  FDM_LAUNCH("k_permute_in");
}

void launch_permute_out(const double* y_tree, const int32_t* perm, int64_t n,
                        double* y_user, hipStream_t s) {
  if (n == 0) return;
  k_permute_out<<<grid_for(n, 256), 256, 0, s>>>(
      reinterpret_cast<const double2*>(y_tree), perm, n, reinterpret_cast<double2*>(y_user));
  FDM_LAUNCH("k_permute_out");
}

void launch_permute_in_c64(const float* v_user, const int32_t* perm, int64_t n,
                           double* v_tree, hipStream_t s) {
  if (n == 0) return;
  k_permute_in_c64<<<grid_for(n, 256), 256, 0, s>>>(
      reinterpret_cast<const float2*>(v_user), perm, n, reinterpret_cast<double2*>(v_tree));
  FDM_LAUNCH("k_permute_in_c64");
}

void launch_permute_out_c64(const double* y_tree, const int32_t* perm, int64_t n,
                            float* y_user, hipStream_t s) {
  if (n == 0) return;
  k_permute_out_c64<<<grid_for(n, 256), 256, 0, s>>>(
      reinterpret_cast<const double2*>(y_tree), perm, n, reinterpret_cast<float2*>(y_user));
  FDM_LAUNCH("k_permute_out_c64");
}

void launch_s2m_boxes(Plan& P, int level, const int32_t* boxes, int64_t nb, hipStream_t s) {
  LevelData& Lp = P.L[level];
  if (nb == 0) return;
  dim3 grid(static_cast<unsigned>(std::min<int64_t>(nb, 1 << 20)), Lp.nd);
  auto pick = [&](auto nper) {
    constexpr int N = decltype(nper)::value;
    return Lp.mom16.get() ? k_s2m<true, N> : k_s2m<false, N>;
  };
  const int nper = (P.ip.K + 63) / 64;
  auto kernel = nper <= 1   ? pick(std::integral_constant<int, 1>{})
                : nper <= 2 ? pick(std::integral_constant<int, 2>{})
                : nper <= 4 ? pick(std::integral_constant<int, 4>{})
                : nper <= 6 ? pick(std::integral_constant<int, 6>{})
                : nper <= 8 ? pick(std::integral_constant<int, 8>{})
                            : pick(std::integral_constant<int, kPerLane>{});
  kernel<<<grid, 64, 0, s>>>(P.S.x.get(), P.S.y.get(), P.S.z.get(),
                             reinterpret_cast<const double2*>(P.vtree()),
                             P.S.key[level].get(), P.S.start[level].get(),
                             P.S.count[level].get(), boxes, nb, level, P.lo[0], P.lo[1],
                             P.lo[2], Lp.hv(), Lp.dirvec.get(), Lp.nd, P.kappa, P.ip,
                             reinterpret_cast<double2*>(Lp.mom64.get()),
                             reinterpret_cast<float2*>(Lp.mom32.get()), Lp.mom16.get());
  FDM_LAUNCH("k_s2m");
}

void launch_s2m(Plan& P, hipStream_t s) {
  launch_s2m_boxes(P, P.levels, nullptr, P.S.nb[P.levels], s);
}

void launch_m2m(Plan& P, int level, hipStream_t s) {
  LevelData& Lc = P.L[level];
  LevelData& L1 = P.L[level + 1];
  const int64_t nb = P.S.nb[level];
  if (nb == 0) return;
  dim3 grid(static_cast<unsigned>(std::min<int64_t>(nb, 1 << 20)), Lc.nd);
  const size_t lds = size_t(6) * P.ip.K * sizeof(double2);
  if (lds <= kOctLds) {  // the eight children together (m <= 7)
    k_m2m_oct<<<grid, kXT, lds, s>>>(
        reinterpret_cast<const double2*>(L1.mom64.get()), L1.nd, P.S.grid[level + 1].get(),
        P.S.key[level].get(), nb, level, L1.hv(), Lc.dirvec.get(), L1.dirvec.get(), Lc.nd,
        P.l_hf, P.kappa, P.ip, reinterpret_cast<double2*>(Lc.mom64.get()),
        reinterpret_cast<float2*>(Lc.mom32.get()), Lc.mom16.get());
    FDM_LAUNCH("k_m2m_oct");
    return;
  }
  k_m2m<<<grid, kXT, 0, s>>>(reinterpret_cast<const double2*>(L1.mom64.get()), L1.nd,
                            P.S.grid[level + 1].get(), P.S.key[level].get(), nb, level,
                            L1.hv(), Lc.dirvec.get(), L1.dirvec.get(), Lc.nd, P.l_hf,
                            P.kappa, P.ip, reinterpret_cast<double2*>(Lc.mom64.get()),
                            reinterpret_cast<float2*>(Lc.mom32.get()), Lc.mom16.get());
  FDM_LAUNCH("k_m2m");
}

}  // namespace fdm
