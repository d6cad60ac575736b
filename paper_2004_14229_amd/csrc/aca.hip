// Low-rank coupling matrices on the device (Sect. 2.7): every stored coupling
// matrix A~ of a plan (one per admissible level and offset) is compressed by
// partially pivoted adaptive cross approximation, A~ ~ sum_l u_l v_l^T, and
// the crosses are written in the layouts the two-stage coupling kernels read
// (m2l_aca.hip):
//   U  (Kp x kp): U(row, l) = u_l[row], k-major, re and im planes (FP32);
//   Vt (kp x Kp): Vt(l, k) = v_l[k],    k-major, re and im planes (FP32);
// so that A~ M = U (Vt M).  Entries of A~ are evaluated where ACA reads them
// (its pivot rows and columns), in FP64, from the same formula as the dense
// bank.
//
// The cross loop is the one of the host fdm_aca (and of the paper's method):
// the pivot row's residual is scaled to 1 at its entry of largest modulus
// (first index on ties), the residual of that column is the next u, the next
// pivot row is the unused row where u is largest, a vanishing residual row
// passes to the first unused row, and the loop stops once |u_k| |v_k| <= eps
// |S_k|_F (the Frobenius norm of the sum so far, updated from inner
// products) or after kp crosses.
#include "plan.hpp"
#include "device_math.hpp"

namespace fdm {

namespace {

constexpr int kAcaThreads = 256;

// Entry (row, col) of the coupling matrix of one (level, offset, direction),
// centre-relative phase form (as in the dense bank).
__device__ __forceinline__ double2 coupling_entry(int row, int col, const BankLevel& L,
                                                  const double o[3], const double c[3],
                                                  const Interp& ip) {
  const int m1 = ip.m1;
  const int a[3] = {row / (m1 * m1), (row / m1) % m1, row % m1};
  const int b[3] = {col / (m1 * m1), (col / m1) % m1, col % m1};
  double d[3], rel[3];
  for (int q = 0; q < 3; ++q) {
    rel[q] = 0.5 * L.h[q] * (ip.node[a[q]] - ip.node[b[q]]);
    d[q] = L.h[q] * o[q] + rel[q];
  }
  const double rr = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
  const double arg = L.kappa * rr - L.kappa * (rel[0] * c[0] + rel[1] * c[1] + rel[2] * c[2]);
  double sn, cs;
  phase_sincos(arg, sn, cs);
  const double w = 1.0 / (4.0 * M_PI * rr);
  return make_double2(cs * w, sn * w);
}

__device__ __forceinline__ double abs2(double2 z) { return z.x * z.x + z.y * z.y; }

// Block-wide arg max of `val` over the threads' candidates (value, index),
// the first index on ties; -1 / -1.0 when no thread has a candidate.
__device__ __forceinline__ void block_argmax(double val, int idx, double* sv, int* si,
                                             double& best, int& at) {
  const int t = threadIdx.x;
  sv[t] = val;
  si[t] = idx;
  __syncthreads();
  for (int s = kAcaThreads / 2; s > 0; s >>= 1) {
    if (t < s) {
      const double v2 = sv[t + s];
      const int i2 = si[t + s];
      if (i2 >= 0 && (si[t] < 0 || v2 > sv[t] || (v2 == sv[t] && i2 < si[t]))) {
        sv[t] = v2;
        si[t] = i2;
      }
    }
    __syncthreads();
  }
  best = sv[0];
  at = si[0];
  __syncthreads();
}

__device__ __forceinline__ double block_sum(double val, double* sv) {
  const int t = threadIdx.x;
  sv[t] = val;
  __syncthreads();
  for (int s = kAcaThreads / 2; s > 0; s >>= 1) {
    if (t < s) sv[t] += sv[t + s];
    __syncthreads();
  }
  const double r = sv[0];
  __syncthreads();
  return r;
}

// One workgroup per matrix of the list (grid-stride); us / vs: FP64 cross
// scratch of kp x K complex per workgroup slot (blockIdx.x).
__global__ void __launch_bounds__(kAcaThreads) k_aca(
    const int32_t* __restrict__ info, int64_t n_mat, const BankLevel* __restrict__ lv,
    Interp ip, double eps, int kp, double2* __restrict__ us_all,
    double2* __restrict__ vs_all, float* __restrict__ bank, int32_t* __restrict__ rank) {
  __shared__ double2 r[kMaxK];
  __shared__ double2 u[kMaxK];
  __shared__ unsigned char used[kMaxK];
  __shared__ double sv[kAcaThreads];
  __shared__ int si[kAcaThreads];
  __shared__ double cross_l[64];
  const int K = ip.K, Kp = ip.Kp, t = threadIdx.x;
  double2* us = us_all + int64_t(blockIdx.x) * kp * K;
  double2* vs = vs_all + int64_t(blockIdx.x) * kp * K;
  const int64_t per = int64_t(Kp) * kp;  // one plane of U or of Vt
  for (int64_t id = blockIdx.x; id < n_mat; id += gridDim.x) {
    const int32_t* in = info + 5 * id;
    const BankLevel L = lv[in[0]];
    const double o[3] = {double(in[1]), double(in[2]), double(in[3])};
    const double c[3] = {L.dirvec[3 * in[4]], L.dirvec[3 * in[4] + 1], L.dirvec[3 * in[4] + 2]};
    for (int q = t; q < K; q += kAcaThreads) used[q] = 0;
    __syncthreads();
    double fro2 = 0.0;
    int k = 0, i = 0;
    while (k < kp) {
      // residual of row i
      for (int j = t; j < K; j += kAcaThreads) {
        double2 z = coupling_entry(i, j, L, o, c, ip);
        for (int l = 0; l < k; ++l) {
          const double2 ul = us[int64_t(l) * K + i], vl = vs[int64_t(l) * K + j];
          z.x -= ul.x * vl.x - ul.y * vl.y;
          z.y -= ul.x * vl.y + ul.y * vl.x;
        }
        r[j] = z;
      }
      if (t == 0) used[i] = 1;
      __syncthreads();
      double bv = -1.0;
      int bj = -1;
      for (int j = t; j < K; j += kAcaThreads) {
        const double a = abs2(r[j]);
        if (a > bv) {
          bv = a;
          bj = j;
        }
      }
      double best;
      int j = 0;
      block_argmax(bv, bj, sv, si, best, j);
      const double2 rj = r[j];
      if (rj.x == 0.0 && rj.y == 0.0) {  // the row is reproduced: first unused row
        int f = K;
        for (int q = t; q < K; q += kAcaThreads)
          if (!used[q]) {
            f = q;
            break;
          }
        double dummy;
        int first = -1;
        block_argmax(f < K ? -double(f) : -1.0, f < K ? f : -1, sv, si, dummy, first);
        if (first < 0) break;
        i = first;
        continue;
      }
      // v = r / r_j; the residual of column j is u
      const double den = abs2(rj);
      double nv2 = 0.0, nu2 = 0.0;
      for (int q = t; q < K; q += kAcaThreads) {
        const double2 z = r[q];
        const double2 v = make_double2((z.x * rj.x + z.y * rj.y) / den,
                                       (z.y * rj.x - z.x * rj.y) / den);
        vs[int64_t(k) * K + q] = v;
        nv2 += abs2(v);
        double2 w = coupling_entry(q, j, L, o, c, ip);
        for (int l = 0; l < k; ++l) {
          const double2 vl = vs[int64_t(l) * K + j], ul = us[int64_t(l) * K + q];
          w.x -= vl.x * ul.x - vl.y * ul.y;
          w.y -= vl.x * ul.y + vl.y * ul.x;
        }
        u[q] = w;
        us[int64_t(k) * K + q] = w;
        nu2 += abs2(w);
      }
      __syncthreads();
      nv2 = block_sum(nv2, sv);
      nu2 = block_sum(nu2, sv);
      // 2 Re sum_l <u_l, u> <v_l, v>: thread l forms the two inner products
      if (t < k) {
        double ur = 0.0, ui = 0.0, vr = 0.0, vi = 0.0;
        for (int q = 0; q < K; ++q) {
          const double2 a = us[int64_t(t) * K + q], b = u[q];
          ur += a.x * b.x + a.y * b.y;
          ui += a.x * b.y - a.y * b.x;
          const double2 p = vs[int64_t(t) * K + q], w = vs[int64_t(k) * K + q];
          vr += p.x * w.x + p.y * w.y;
          vi += p.x * w.y - p.y * w.x;
        }
        cross_l[t] = ur * vr - ui * vi;
      }
      __syncthreads();
      double cross = 0.0;
      for (int l = 0; l < k; ++l) cross += cross_l[l];  // in order of l, every thread
      const double nu = sqrt(nu2), nv = sqrt(nv2);
      fro2 += 2.0 * cross + (nu * nv) * (nu * nv);
      ++k;
      if (nu * nv <= eps * sqrt(fmax(fro2, 0.0))) break;
      // next pivot row: the unused row where u is largest
      bv = -1.0;
      bj = -1;
      for (int q = t; q < K; q += kAcaThreads) {
        if (used[q]) continue;
        const double a = abs2(u[q]);
        if (a > bv) {
          bv = a;
          bj = q;
        }
      }
      int next = -1;
      block_argmax(bv, bj, sv, si, best, next);
      if (next < 0) break;
      i = next;
    }
    // FP32 factors in the kernels' layouts, zero beyond the rank and K
    float* Ub = bank + id * 4 * per;
    float* Vb = Ub + 2 * per;
    for (int e = t; e < Kp * kp; e += kAcaThreads) {
      const int l = e / Kp, row = e % Kp;  // U(row, l) at l * Kp + row
      double2 z = make_double2(0.0, 0.0);
      if (l < k && row < K) z = us[int64_t(l) * K + row];
      Ub[e] = float(z.x);
      Ub[per + e] = float(z.y);
      const int kk = e / kp, l2 = e % kp;  // Vt(l, k) at k * kp + l
      double2 w = make_double2(0.0, 0.0);
      if (l2 < k && kk < K) w = vs[int64_t(l2) * K + kk];
      Vb[e] = float(w.x);
      Vb[per + e] = float(w.y);
    }
    if (t == 0) rank[id] = k;
    __syncthreads();
  }
}

}  // namespace

int64_t aca_matrix_bytes(const Interp& ip, int kp) { return int64_t(4) * ip.Kp * kp * 4; }

void launch_aca(const int32_t* info, int64_t n_mat, const BankLevel* lv, const Interp& ip,
                double eps, int kp, float* bank, int32_t* rank, hipStream_t s) {
  if (n_mat == 0) return;
  if (kp > 64 || kp < 1) fail(FDM_ERR_INVALID_ARG, "ACA rank cap must be in 1..64");
  // cross scratch for a bounded number of concurrent matrices
  const int64_t slots = std::min<int64_t>(n_mat, 4096);
  DevBuf<double2> us(size_t(slots) * kp * ip.K), vs(size_t(slots) * kp * ip.K);
  k_aca<<<static_cast<unsigned>(slots), kAcaThreads, 0, s>>>(
      info, n_mat, lv, ip, eps, kp, us.get(), vs.get(), bank, rank);
  FDM_LAUNCH("k_aca");
  FDM_HIP(hipStreamSynchronize(s));  // scratch freed on return
}

}  // namespace fdm
