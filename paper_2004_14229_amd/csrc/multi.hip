// Several right-hand sides on one plan, Y = A~ V (repeated application of
// the same operator, Sect. 4): everything the plan built (trees, work
// lists, the coupling bank or its low-rank factors) serves every vector,
// and the near field evaluates each kernel value f(x_j, y_k) once for up to
// four vectors (the near field's cost is the kernel evaluation: a square
// root, a reciprocal and a reduced sine/cosine per pair).  The far field
// runs vector by vector through the plan's own phases and launches, so each
// result equals that of fdm_plan_matvec on the same vector bit for bit.
#include "plan.hpp"
#include "nearfield.hpp"
#include "capi.hpp"

namespace fdm {

namespace {

constexpr int kMaxR = 4;  // vectors per near-field pass

// Thread per target point: the near field of R vectors (tree order, vector
// q at vm + q * nS), in the summation order of the one-vector kernels.
template <int R>
__global__ void __launch_bounds__(256) k_p2p_multi(P2PDesc d, int64_t nT,
                                                   const double2* __restrict__ vm, int64_t nS,
                                                   double2* __restrict__ ym) {
  const int64_t j = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  if (j >= nT) return;
  const double px = d.xt[j], py = d.yt[j], pz = d.zt[j];
  int ix, iy, iz;
  demorton3(d.keyT[d.leaf_of[j]], d.level, ix, iy, iz);
  const int lim = 1 << d.level;
  double ar[R], ai[R];
#pragma unroll
  for (int q = 0; q < R; ++q) ar[q] = ai[q] = 0.0;
  for (int o = 0; o < d.n_off; ++o) {
    const int sx = ix - d.near_off[3 * o], sy = iy - d.near_off[3 * o + 1],
              sz = iz - d.near_off[3 * o + 2];
    if (sx < 0 || sy < 0 || sz < 0 || sx >= lim || sy >= lim || sz >= lim) continue;
    const int32_t sb = d.gridS[morton3(sx, sy, sz, d.level)];
    if (sb < 0) continue;
    const int k0 = d.startS[sb], kn = d.countS[sb];
    for (int k = k0; k < k0 + kn; ++k) {
      double fr, fi;
      if (!kernel_value(px, py, pz, d.xs[k], d.ys[k], d.zs[k], d.kappa, fr, fi)) continue;
#pragma unroll
      for (int q = 0; q < R; ++q) kernel_accumulate(fr, fi, vm[q * nS + k], ar[q], ai[q]);
    }
  }
#pragma unroll
  for (int q = 0; q < R; ++q) ym[q * nT + j] = make_double2(ar[q], ai[q]);
}

void launch_p2p_multi(Plan& P, const double* vm, double* ym, int nv, hipStream_t s) {
  const unsigned grid = static_cast<unsigned>((P.nT + 255) / 256);
  const P2PDesc d = p2p_desc(P);
  auto* v2 = reinterpret_cast<const double2*>(vm);
  auto* y2 = reinterpret_cast<double2*>(ym);
  switch (nv) {
    case 1: k_p2p_multi<1><<<grid, 256, 0, s>>>(d, P.nT, v2, P.nS, y2); break;
    case 2: k_p2p_multi<2><<<grid, 256, 0, s>>>(d, P.nT, v2, P.nS, y2); break;
    case 3: k_p2p_multi<3><<<grid, 256, 0, s>>>(d, P.nT, v2, P.nS, y2); break;
    default: k_p2p_multi<4><<<grid, 256, 0, s>>>(d, P.nT, v2, P.nS, y2); break;
  }
  FDM_LAUNCH("k_p2p_multi");
}

// Restores the plan's own tree-order vectors when a pass ends or fails.
struct ViewGuard {
  Plan& P;
  ~ViewGuard() {
    P.v_view = nullptr;
    P.y_view = nullptr;
  }
};

}  // namespace

}  // namespace fdm

using namespace fdm;

extern "C" int fdm_plan_matvec_multi(fdm_plan* plan, const void* V, void* Y, int nrhs, int c64,
                                     void* stream) {
  return guarded([&] {
    if (!plan) fail(FDM_ERR_INVALID_ARG, "plan is NULL");
    Plan& P = plan->p;
    if (nrhs < 1) fail(FDM_ERR_INVALID_ARG, "nrhs must be >= 1");
    if (c64 != 0 && c64 != 1) fail(FDM_ERR_INVALID_ARG, "c64 must be 0 or 1");
    if (P.batch_owner) fail(FDM_ERR_STATE, "the plan belongs to a batch");
    const int64_t w = c64 ? 8 : 16;
    if (P.nS) check_device_ptr(V, "V");
    if (P.nT) check_device_ptr(Y, "Y");
    if (P.nS && P.nT) {
      const char* a = static_cast<const char*>(V);
      const char* b = static_cast<const char*>(Y);
      if (a < b + w * P.nT * nrhs && b < a + w * P.nS * nrhs)
        fail(FDM_ERR_INVALID_ARG, "V and Y overlap");
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    auto vin = [&](int r) { return static_cast<const char*>(V) + w * P.nS * r; };
    auto yout = [&](int r) { return static_cast<char*>(Y) + w * P.nT * r; };
    if (P.nT == 0) return;
    if (P.nS == 0 || p2p_queued(P, P.tune)) {  // (near field inside the coupling queue)
      for (int r = 0; r < nrhs; ++r) plan_matvec(P, vin(r), yout(r), c64 != 0, s);
      return;
    }
    if (!P.sched_ready) build_plan_schedule(P, s);
    if (P.vm_tree.size() < size_t(2 * P.nS * nrhs)) P.vm_tree.alloc(2 * P.nS * nrhs, &P.tally);
    if (P.ym_tree.size() < size_t(2 * P.nT * nrhs)) P.ym_tree.alloc(2 * P.nT * nrhs, &P.tally);
    double* vm = P.vm_tree.get();
    double* ym = P.ym_tree.get();
    for (int r = 0; r < nrhs; ++r) {
      if (c64)
        launch_permute_in_c64(reinterpret_cast<const float*>(vin(r)), P.S.perm.get(), P.nS,
                              vm + 2 * P.nS * r, s);
      else
        launch_permute_in(reinterpret_cast<const double*>(vin(r)), P.S.perm.get(), P.nS,
                          vm + 2 * P.nS * r, s);
    }
    ViewGuard guard{P};
    // near field, stored first
    if (P.adaptive()) {
      for (int r = 0; r < nrhs; ++r) {
        P.v_view = vm + 2 * P.nS * r;
        P.y_view = ym + 2 * P.nT * r;
        launch_p2p(P, s);
      }
    } else {
      for (int r = 0; r < nrhs; r += kMaxR)
        launch_p2p_multi(P, vm + 2 * P.nS * r, ym + 2 * P.nT * r, std::min(kMaxR, nrhs - r), s);
    }
    // far field, added, vector by vector
    const int p = P.levels;
    for (int r = 0; r < nrhs; ++r) {
      P.v_view = vm + 2 * P.nS * r;
      P.y_view = ym + 2 * P.nT * r;
      if (P.l_min <= p) {
        launch_s2m(P, s);
        for (int l = p - 1; l >= P.l_min; --l) plan_m2m_level(P, l, s);
      }
      run_schedule(P.sched, P.heads.get(), P.prec, P.ip, P.tune, s);
      if (P.l_min <= p)
        for (int l = P.l_min; l < p; ++l) launch_l2l(P, l, s);
      launch_l2t(P, s);
      if (c64)
        launch_permute_out_c64(P.ytree(), P.T.perm.get(), P.nT, reinterpret_cast<float*>(yout(r)),
                               s);
      else
        launch_permute_out(P.ytree(), P.T.perm.get(), P.nT, reinterpret_cast<double*>(yout(r)), s);
    }
    P.has_run = true;
  });
}
