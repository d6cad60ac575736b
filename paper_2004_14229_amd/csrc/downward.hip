// Backward transformation of Alg. 4 (Sect. 2.6) in the centre-relative
// phase form:
//
//   L2L  g~_{t',c'} = G_{t',c'} + sum_{c : dir_(l+1)(c) = c'} E~d_{t',c} .* (E_{t'} g~_{t,c})
//   L2T  y_j += sum_c sum_nu L_{t,nu}(x_j) exp(i kappa <x_j - m_t, c>) g~_{t,c}[nu]
//
// with G the coupling (M2L) result of the box and E~d as in the forward
// transformation.  One workgroup owns one (box, direction) local, so every
// local is written exactly once per level, with a fixed order of the sums.
#include "plan.hpp"
#include "device_math.hpp"

namespace fdm {

namespace {

template <class GT>
__device__ __forceinline__ double2 load_c(const GT* p, int64_t i);
template <>
__device__ __forceinline__ double2 load_c<double2>(const double2* p, int64_t i) {
  return p[i];
}
template <>
__device__ __forceinline__ double2 load_c<float2>(const float2* p, int64_t i) {
  float2 v = p[i];
  return make_double2(v.x, v.y);
}

// One workgroup (kXT threads) per (child box t' on level l+1, direction c').
template <class GT>
__global__ void __launch_bounds__(kXT) k_l2l(
    const double2* __restrict__ ploc, int nd, const int32_t* __restrict__ pgrid,
    const uint32_t* __restrict__ key1, int64_t nb1, int level, double3 h1,
    const double* __restrict__ dirvec, const double* __restrict__ dirvec1, int nd1,
    int l_hf, double kappa, Interp ip, const GT* g_m2l,
    double2* loc1) {  // g_m2l may alias loc1 (read before write, same thread)
  __shared__ double2 buf[2][kMaxK];
  __shared__ double2 ph[3][kMaxM1];
  const int lane = threadIdx.x;
  const int cp = blockIdx.y;  // c' on level l+1
  const int m1 = ip.m1, K = ip.K, Kp = ip.Kp;
  // parent directions c with dir_(l+1)(c) = c'
  const bool hf_child = level + 1 <= l_hf;
  const int c_begin = hf_child ? 4 * cp : 0;
  const int c_end = hf_child ? 4 * cp + 4 : nd;
  const double cv1[3] = {dirvec1[3 * cp], dirvec1[3 * cp + 1], dirvec1[3 * cp + 2]};
  for (int64_t b = blockIdx.x; b < nb1; b += gridDim.x) {
    const uint32_t k1 = key1[b];
    const int32_t par = pgrid[k1 >> 3];
    const int q = k1 & 7;
    const int bq[3] = {(q >> 2) & 1, (q >> 1) & 1, q & 1};
    double2 acc[kPerXT];
    const int64_t obase = (b * nd1 + cp) * int64_t(Kp);
#pragma unroll
    for (int i = 0; i < kPerXT; ++i) {
      const int k = lane + kXT * i;
      acc[i] = k < K ? load_c(g_m2l, obase + k) : make_double2(0.0, 0.0);
    }
    for (int c = c_begin; c < c_end; ++c) {
      const double cv[3] = {dirvec[3 * c], dirvec[3 * c + 1], dirvec[3 * c + 2]};
      __syncthreads();
      if (lane < 3 * m1) {
        const int d = lane / m1, nu = lane % m1;
        const double hd = d == 0 ? h1.x : d == 1 ? h1.y : h1.z;
        const double r = 0.5 * hd * ip.node[nu];  // xi - m_{t'}
        const double off = (bq[d] - 0.5) * hd;    // m_{t'} - m_t
        double sn, cs;
        phase_sincos(kappa * ((r + off) * cv[d] - r * cv1[d]), sn, cs);
        ph[d][nu] = make_double2(cs, sn);
      }
      const double2* src = ploc + (int64_t(par) * nd + c) * Kp;
      for (int k = lane; k < K; k += kXT) buf[0][k] = src[k];
      __syncthreads();
      apply_transfer(buf, ip, bq, false, lane, kXT);  // buf[1] = E_{t'} g
#pragma unroll
      for (int i = 0; i < kPerXT; ++i) {
        const int k = lane + kXT * i;
        if (k < K) {
          const int n3 = k % m1, n2 = (k / m1) % m1, n1 = k / (m1 * m1);
          const double2 f = cmul(cmul(ph[0][n1], ph[1][n2]), ph[2][n3]);
          const double2 v = cmul(f, buf[1][k]);
          acc[i].x += v.x;
          acc[i].y += v.y;
        }
      }
    }
#pragma unroll
    for (int i = 0; i < kPerXT + 1; ++i) {
      const int k = lane + kXT * i;
      if (k < Kp) loc1[obase + k] = (k < K && i < kPerXT) ? acc[i < kPerXT ? i : 0]
                                                         : make_double2(0.0, 0.0);
    }
  }
}

// One workgroup (kXT threads) per (parent box t, direction c' of the
// children's level, x half bx), the four children of that half together.
// For each parent direction c with dir_(l+1)(c) = c', the x pass of E_{t'}
// takes the parent's local to its bx half, the y pass that to the two
// (bx, by) quarters and the z pass to the four children, each then
// multiplied by its phase factors and added to the child's local: 7
// one-dimensional passes per workgroup and c (14 per parent, against 24
// child by child) and 3 barriers.  The phase factors depend only on c and
// the child's octant bit per axis and are formed once per workgroup.  The
// children's locals start from their coupling results and stay with the
// thread that writes them.  Needs K <= 512 (m <= 7); dynamic LDS: 4 K
// complex values.
constexpr int kL2lMaxC = 6;  // parent directions c per c' (6 on the level l_hf)
constexpr int kPerXT4 = (4 * 512 + kXT - 1) / kXT;

template <class GT>
__global__ void __launch_bounds__(kXT) k_l2l_oct(
    const double2* __restrict__ ploc, int nd, const uint32_t* __restrict__ key, int64_t nb,
    const int32_t* __restrict__ grid1, int level, double3 h1,
    const double* __restrict__ dirvec, const double* __restrict__ dirvec1, int nd1,
    int l_hf, double kappa, Interp ip, const GT* g_m2l,
    double2* loc1) {  // g_m2l may alias loc1 (read before write, same thread)
  extern __shared__ double2 smem[];
  __shared__ double2 ph[kL2lMaxC][3][2][kMaxM1];  // c, axis, octant bit, node
  __shared__ double e1[2][kMaxM1][kMaxM1];         // E1[b][j][k]
  __shared__ int32_t chs[4];
  const int lane = threadIdx.x;
  const int cp = blockIdx.y;  // c' on level l+1
  const int bx = blockIdx.z;  // the children's x bit
  const int m1 = ip.m1, m2 = m1 * m1, K = ip.K, Kp = ip.Kp;
  double2* par = smem;         // [K]: the parent's local for c
  double2* xh = smem + K;      // [K]: after the x pass (half bx)
  double2* yq = smem + 2 * K;  // [2][K]: after the y pass (by)
  const bool hf_child = level + 1 <= l_hf;
  const int c_begin = hf_child ? 4 * cp : 0;
  const int nc = hf_child ? 4 : nd;
  for (int e = lane; e < nc * 6 * m1; e += kXT) {  // E~d_{t',c} per axis
    const int ci = e / (6 * m1), d = (e / (2 * m1)) % 3, b = (e / m1) % 2, nu = e % m1;
    const int c = c_begin + ci;
    const double hd = d == 0 ? h1.x : d == 1 ? h1.y : h1.z;
    const double r = 0.5 * hd * ip.node[nu];  // xi - m_{t'}
    const double off = (b - 0.5) * hd;        // m_{t'} - m_t
    double sn, cs;
    phase_sincos(kappa * ((r + off) * dirvec[3 * c + d] - r * dirvec1[3 * cp + d]), sn, cs);
    ph[ci][d][b][nu] = make_double2(cs, sn);
  }
  for (int e = lane; e < 2 * m2; e += kXT) {
    const int b = e / m2, j = (e / m1) % m1, k = e % m1;
    e1[b][j][k] = ip.E1[b][j][k];
  }
  for (int64_t t = blockIdx.x; t < nb; t += gridDim.x) {
    __syncthreads();  // (tables; the previous box's reads of chs)
    if (lane < 4) chs[lane] = grid1[(key[t] << 3) | (4 * bx + lane)];
    __syncthreads();
    if (max(max(chs[0], chs[1]), max(chs[2], chs[3])) < 0) continue;  // no child here
    double2 acc[kPerXT4];
#pragma unroll
    for (int i = 0; i < kPerXT4; ++i) {
      const int e = lane + kXT * i;
      acc[i] = make_double2(0.0, 0.0);
      if (e < 4 * K) {
        const int q = e / K, k = e - q * K;  // q = 2 by + bz
        const int32_t ch = chs[q];
        if (ch >= 0) acc[i] = load_c(g_m2l, (int64_t(ch) * nd1 + cp) * Kp + k);
      }
    }
    for (int ci = 0; ci < nc; ++ci) {
      const double2* src = ploc + (t * nd + c_begin + ci) * int64_t(Kp);
      for (int k = lane; k < K; k += kXT) par[k] = src[k];
      __syncthreads();
      for (int e = lane; e < K; e += kXT) {  // x pass (stride m1^2), half bx
        const int j = e / m2, base = e - j * m2;
        double re = 0.0, im = 0.0;
        for (int k = 0; k < m1; ++k) {
          const double w = e1[bx][j][k];
          re += w * par[base + k * m2].x;
          im += w * par[base + k * m2].y;
        }
        xh[e] = make_double2(re, im);
      }
      __syncthreads();
      for (int e = lane; e < 2 * K; e += kXT) {  // y pass (stride m1)
        const int by = e / K, ee = e - by * K;
        const int j = (ee / m1) % m1, base = ee - j * m1;
        double re = 0.0, im = 0.0;
        for (int k = 0; k < m1; ++k) {
          const double w = e1[by][j][k];
          re += w * xh[base + k * m1].x;
          im += w * xh[base + k * m1].y;
        }
        yq[e] = make_double2(re, im);
      }
      __syncthreads();
#pragma unroll
      for (int i = 0; i < kPerXT4; ++i) {  // z pass (stride 1), phase, into the child
        const int e = lane + kXT * i;
        if (e < 4 * K) {
          const int q = e / K, k = e - q * K;  // q = 2 by + bz
          if (chs[q] >= 0) {
            const int j = k % m1, base = k - j;
            const double2* y = yq + (q >> 1) * K + base;
            double re = 0.0, im = 0.0;
            for (int kk = 0; kk < m1; ++kk) {
              const double w = e1[q & 1][j][kk];
              re += w * y[kk].x;
              im += w * y[kk].y;
            }
            const int n1 = k / m2, n2 = (k / m1) % m1, n3 = k % m1;
            const double2 f = cmul(cmul(ph[ci][0][bx][n1], ph[ci][1][q >> 1][n2]),
                                   ph[ci][2][q & 1][n3]);
            const double2 v = cmul(f, make_double2(re, im));
            acc[i].x += v.x;
            acc[i].y += v.y;
          }
        }
      }
      // (the next direction's load writes par only; xh and yq are rewritten
      // after the barrier that follows it)
    }
#pragma unroll
    for (int i = 0; i < kPerXT4; ++i) {
      const int e = lane + kXT * i;
      if (e < 4 * K) {
        const int q = e / K, k = e - q * K;
        const int32_t ch = chs[q];
        if (ch >= 0) loc1[(int64_t(ch) * nd1 + cp) * Kp + k] = acc[i];
      }
    }
    for (int e = lane; e < 4 * (Kp - K); e += kXT) {  // zero padding
      const int q = e / (Kp - K), k = K + e % (Kp - K);
      const int32_t ch = chs[q];
      if (ch >= 0) loc1[(int64_t(ch) * nd1 + cp) * Kp + k] = make_double2(0.0, 0.0);
    }
  }
}

// One wave per leaf box: every point of the box, every direction.
// NPER: coefficients per lane, ceil(K / 64) (registers scale with it).
template <int NPER>
__global__ void __launch_bounds__(64) k_l2t(
    const double* __restrict__ x, const double* __restrict__ y,
    const double* __restrict__ z, const uint32_t* __restrict__ key,
    const int32_t* __restrict__ start, const int32_t* __restrict__ count,
    const int32_t* __restrict__ boxes, int64_t nb,
    int level, double lo0, double lo1, double lo2, double3 h,
    const double* __restrict__ dirvec, int nd, double kappa, Interp ip,
    const double2* __restrict__ loc, double2* __restrict__ y_tree) {
  __shared__ double lag[3][kMaxM1];
  const int lane = threadIdx.x;
  const int m1 = ip.m1, K = ip.K, Kp = ip.Kp;
  for (int64_t bi = blockIdx.x; bi < nb; bi += gridDim.x) {
    const int64_t b = boxes ? boxes[bi] : bi;
    int ix, iy, iz;
    demorton3(key[b], level, ix, iy, iz);
    const double mx = lo0 + (ix + 0.5) * h.x, my = lo1 + (iy + 0.5) * h.y,
                 mz = lo2 + (iz + 0.5) * h.z;
    const double inv_half[3] = {2.0 / h.x, 2.0 / h.y, 2.0 / h.z};
    const int p0 = start[b], pn = count[b];
    // one direction (every level below the high-frequency ones): the box's
    // local is read once, before the first point's barriers
    double2 g0[NPER];
    if (nd == 1) {
#pragma unroll
      for (int i = 0; i < NPER; ++i) {
        const int k = lane + 64 * i;
        g0[i] = k < K ? loc[b * int64_t(Kp) + k] : make_double2(0.0, 0.0);
      }
    }
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
      double yr = 0.0, yi = 0.0;
      for (int c = 0; c < nd; ++c) {
        const double2* g = loc + (b * nd + c) * int64_t(Kp);
        double sr = 0.0, si = 0.0;
#pragma unroll
        for (int i = 0; i < NPER; ++i) {
          const int k = lane + 64 * i;
          if (k < K) {
            const int n3 = k % m1, n2 = (k / m1) % m1, n1 = k / (m1 * m1);
            const double L = lag[0][n1] * lag[1][n2] * lag[2][n3];
            const double2 gv = nd == 1 ? g0[i] : g[k];
            sr += L * gv.x;
            si += L * gv.y;
          }
        }
        for (int off = 32; off > 0; off >>= 1) {
          sr += __shfl_xor(sr, off, 64);
          si += __shfl_xor(si, off, 64);
        }
        const double cx = dirvec[3 * c], cy = dirvec[3 * c + 1], cz = dirvec[3 * c + 2];
        double sn, cs;
        phase_sincos(kappa * (dx * cx + dy * cy + dz * cz), sn, cs);
        yr += cs * sr - sn * si;
        yi += cs * si + sn * sr;
      }
      if (lane == 0) {  // added to the near field stored before
        const double2 yn = y_tree[j];
        y_tree[j] = make_double2(yn.x + yr, yn.y + yi);
      }
    }
  }
}

__global__ void k_zero_c128(double2* p, int64_t n) {
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * blockDim.x)
    p[i] = make_double2(0.0, 0.0);
}

}  // namespace

void launch_zero_c128(double* p, int64_t n, hipStream_t s) {
  if (n == 0) return;
  k_zero_c128<<<grid_for(n, 256), 256, 0, s>>>(reinterpret_cast<double2*>(p), n);
  FDM_LAUNCH("k_zero_c128");
}

void launch_l2l(Plan& P, int level, hipStream_t s) {
  LevelData& Lc = P.L[level];
  LevelData& L1 = P.L[level + 1];
  const int64_t nb1 = P.T.nb[level + 1];
  if (nb1 == 0) return;
  const int nc = level + 1 <= P.l_hf ? 4 : Lc.nd;  // parent directions per c'
  const size_t lds = size_t(4) * P.ip.K * sizeof(double2);
  if (P.ip.K <= 512 && lds <= kOctLds && nc <= kL2lMaxC) {  // four children together
    const int64_t nb = P.T.nb[level];
    dim3 grid(static_cast<unsigned>(std::min<int64_t>(nb, 1 << 20)), L1.nd, 2);
    k_l2l_oct<double2><<<grid, kXT, lds, s>>>(
        reinterpret_cast<const double2*>(Lc.loc64.get()), Lc.nd, P.T.key[level].get(), nb,
        P.T.grid[level + 1].get(), level, L1.hv(), Lc.dirvec.get(), L1.dirvec.get(), L1.nd,
        P.l_hf, P.kappa, P.ip, reinterpret_cast<const double2*>(L1.loc64.get()),
        reinterpret_cast<double2*>(L1.loc64.get()));
    FDM_LAUNCH("k_l2l_oct");
    return;
  }
  dim3 grid(static_cast<unsigned>(std::min<int64_t>(nb1, 1 << 20)), L1.nd);
  k_l2l<double2><<<grid, kXT, 0, s>>>(
      reinterpret_cast<const double2*>(Lc.loc64.get()), Lc.nd, P.T.grid[level].get(),
      P.T.key[level + 1].get(), nb1, level, L1.hv(), Lc.dirvec.get(), L1.dirvec.get(),
      L1.nd, P.l_hf, P.kappa, P.ip, reinterpret_cast<const double2*>(L1.loc64.get()),
      reinterpret_cast<double2*>(L1.loc64.get()));
  FDM_LAUNCH("k_l2l");
}

void launch_l2t_boxes(Plan& P, int level, const int32_t* boxes, int64_t nb, hipStream_t s) {
  if (P.nT == 0 || nb == 0) return;
  if (level < P.l_min) return;  // no coupling on or above it: the far field is zero
  LevelData& Lp = P.L[level];
  const int nper = (P.ip.K + 63) / 64;
  auto kernel = nper <= 1   ? k_l2t<1>
                : nper <= 2 ? k_l2t<2>
                : nper <= 4 ? k_l2t<4>
                : nper <= 6 ? k_l2t<6>
                : nper <= 8 ? k_l2t<8>
                            : k_l2t<kPerLane>;
  kernel<<<static_cast<unsigned>(std::min<int64_t>(nb, 1 << 20)), 64, 0, s>>>(
      P.T.x.get(), P.T.y.get(), P.T.z.get(), P.T.key[level].get(), P.T.start[level].get(),
      P.T.count[level].get(), boxes, nb, level, P.lo[0], P.lo[1], P.lo[2], Lp.hv(),
      Lp.dirvec.get(), Lp.nd, P.kappa, P.ip, reinterpret_cast<const double2*>(Lp.loc64.get()),
      reinterpret_cast<double2*>(P.ytree()));
  FDM_LAUNCH("k_l2t");
}

void launch_l2t(Plan& P, hipStream_t s) {
  const int p = P.levels;
  if (!P.adaptive()) {
    launch_l2t_boxes(P, p, nullptr, P.T.nb[p], s);
    return;
  }
  // adaptive trees: the leaves of every level, last level first
  launch_l2t_boxes(P, p, P.leafT[p].get(), P.n_leafT[p], s);
  for (int l = 0; l < p; ++l) launch_l2t_boxes(P, l, P.leafT[l].get(), P.n_leafT[l], s);
}

}  // namespace fdm
