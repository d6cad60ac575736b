// Plan construction, the matvec driver of Alg. 4, and the C ABI (fdm.h).
#include "plan.hpp"
#include "capi.hpp"

#include <chrono>
#include <cmath>
#include <cstdio>
#include <set>

namespace fdm {

namespace {

thread_local std::string g_last_error;

Interp make_interp(int m) {
  Interp ip{};
  ip.m1 = m + 1;
  ip.K = ip.m1 * ip.m1 * ip.m1;
  ip.Kp = (ip.K + 31) / 32 * 32;
  for (int nu = 0; nu < ip.m1; ++nu)
    ip.node[nu] = std::cos((2.0 * (nu + 1) - 1.0) * M_PI / (2.0 * ip.m1));
  for (int nu = 0; nu < ip.m1; ++nu) {
    double d = 1.0;
    for (int mu = 0; mu < ip.m1; ++mu)
      if (mu != nu) d *= ip.node[nu] - ip.node[mu];
    ip.wgt[nu] = 1.0 / d;
  }
  // E1[b][j][k] = l_k(child node j in parent reference coordinates)
  for (int b = 0; b < 2; ++b)
    for (int j = 0; j < ip.m1; ++j) {
      const double u = 0.5 * (ip.node[j] + (2 * b - 1));
      for (int k = 0; k < ip.m1; ++k) {
        double p = ip.wgt[k];
        for (int mu = 0; mu < ip.m1; ++mu)
          if (mu != k) p *= u - ip.node[mu];
        ip.E1[b][j][k] = p;
      }
    }
  return ip;
}

}  // namespace

void plan_build(Plan& P, const double* pT, const double* pS, hipStream_t s) {
  auto t0 = std::chrono::steady_clock::now();
  P.ip = make_interp(P.m);
  const double sidev[3] = {P.hi[0] - P.lo[0], P.hi[1] - P.lo[1], P.hi[2] - P.lo[2]};
  P.side = std::max(sidev[0], std::max(sidev[1], sidev[2]));  // the longest side
  build_tree(pT, P.nT, P.lo, P.hi, P.levels, s, &P.tally, P.T);
  build_tree(pS, P.nS, P.lo, P.hi, P.levels, s, &P.tally, P.S);
  if (P.l_hf == -2) {
    P.l_hf = -1;
    for (int l = 0; l <= P.levels; ++l)
      if (P.kappa * (P.side * std::ldexp(1.0, -l)) >= 3.2) P.l_hf = l;
  }
  P.tab = build_level_tables(P.kappa, sidev, P.levels, P.l_hf, P.eta2);
  if (P.adaptive()) build_adaptive(P, s);
  P.l_min = P.levels + 1;
  for (int l = 0; l <= P.levels; ++l)
    if (!P.tab[l].adm.empty()) {
      P.l_min = l;
      break;
    }
  if (P.nT == 0 || P.nS == 0) P.l_min = P.levels + 1;
  P.L.clear();
  P.L.resize(P.levels + 1);
  P.n_bank = 0;
  const int Kp = P.ip.Kp;
  const bool mixed = P.prec != FDM_PREC_FP64;
  for (int l = 0; l <= P.levels; ++l) {
    LevelData& Ld = P.L[l];
    Ld.level = l;
    Ld.nd = direction_count(l, P.l_hf);
    for (int d = 0; d < 3; ++d) Ld.h[d] = sidev[d] * std::ldexp(1.0, -l);
    to_device(Ld.dirvec, direction_vectors(l, P.l_hf), s, &P.tally);
    Ld.bank_base = P.n_bank;
    if (l >= P.l_min) {
      P.n_bank += static_cast<int64_t>(P.tab[l].adm.size());
      const int64_t ns = P.S.nb[l] * int64_t(Ld.nd) * Kp;
      const int64_t nt = P.T.nb[l] * int64_t(Ld.nd) * Kp;
      Ld.mom64.alloc(2 * ns, &P.tally);
      Ld.loc64.alloc(2 * nt, &P.tally);
      if (P.prec == FDM_PREC_BF16X6)
        Ld.mom16.alloc(6 * ns, &P.tally);
      else if (mixed)
        Ld.mom32.alloc(2 * ns, &P.tally);
    }
  }
  // near-field offsets on the leaf level
  {
    const auto& in = P.tab[P.levels].inadm;
    std::vector<int32_t> no;
    for (const Off& o : in) {
      no.push_back(o.x);
      no.push_back(o.y);
      no.push_back(o.z);
    }
    P.n_near_off = static_cast<int>(in.size());
    to_device(P.near_off, no, s, &P.tally);
  }
  P.v_tree.alloc(2 * std::max<int64_t>(P.nS, 1), &P.tally);
  P.y_tree.alloc(2 * std::max<int64_t>(P.nT, 1), &P.tally);
  if (P.l_min <= P.levels) {
    launch_bank(P, s);
    build_m2l_work(P, s);
  }
  // near-field statistics (host, from box counts)
  if (P.adaptive()) {
    adaptive_near_field(P, s);
  } else {
    const int p = P.levels;
    P.near_pairs = 0;
    P.near_entries = 0;
    if (P.nT && P.nS) {
      std::vector<uint32_t> kT = to_host(P.T.key[p].get(), P.T.nb[p], s);
      std::vector<int32_t> cT = to_host(P.T.count[p].get(), P.T.nb[p], s);
      std::vector<int32_t> gS = to_host(P.S.grid[p].get(), size_t(1) << (3 * p), s);
      std::vector<int32_t> cS = to_host(P.S.count[p].get(), P.S.nb[p], s);
      const int lim = 1 << p;
      for (size_t b = 0; b < kT.size(); ++b) {
        int ix, iy, iz;
        demorton3(kT[b], p, ix, iy, iz);
        for (const Off& o : P.tab[p].inadm) {
          int sx = ix - o.x, sy = iy - o.y, sz = iz - o.z;
          if (sx < 0 || sy < 0 || sz < 0 || sx >= lim || sy >= lim || sz >= lim) continue;
          int32_t sb = gS[morton3(sx, sy, sz, p)];
          if (sb < 0) continue;
          P.near_pairs += 1;
          P.near_entries += int64_t(cT[b]) * cS[sb];
        }
      }
    }
  }
  FDM_HIP(hipStreamSynchronize(s));
  P.setup_ms = std::chrono::duration<double, std::milli>(
                   std::chrono::steady_clock::now() - t0).count();
}

// Moments of one level below the last: M2M from the children, then, for an
// adaptive tree, S2M of the level's leaves (whose children are pruned).
void plan_m2m_level(Plan& P, int l, hipStream_t s) {
  launch_m2m(P, l, s);
  if (P.adaptive()) launch_s2m_boxes(P, l, P.leafS[l].get(), P.n_leafS[l], s);
}

// The near field runs as its own launch unless its items share the
// coupling queue (uniform trees only: the queued items read one level).
bool p2p_queued(const Plan& P, const TuneConfig& t) {
  return t.p2p_in_queue && p2p_queue_supported(P.prec, P.ip.Kp) && !P.adaptive() && !P.aca_kp;
}

// Forward pass of one plan: user v -> tree order, S2M, M2M.
void plan_upward(Plan& P, const void* v_user, bool c64, hipStream_t s) {
  if (c64)
    launch_permute_in_c64(static_cast<const float*>(v_user), P.S.perm.get(), P.nS,
                          P.v_tree.get(), s);
  else
    launch_permute_in(static_cast<const double*>(v_user), P.S.perm.get(), P.nS,
                      P.v_tree.get(), s);
  if (P.l_min <= P.levels) {
    launch_s2m(P, s);
    for (int l = P.levels - 1; l >= P.l_min; --l) plan_m2m_level(P, l, s);
  }
}

// Backward pass of one plan: L2L, L2T (added to the near field already in
// y_tree), tree order -> user y.
void plan_downward(Plan& P, void* y_user, bool c64, hipStream_t s) {
  if (P.l_min <= P.levels)
    for (int l = P.l_min; l < P.levels; ++l) launch_l2l(P, l, s);
  launch_l2t(P, s);
  if (c64)
    launch_permute_out_c64(P.y_tree.get(), P.T.perm.get(), P.nT, static_cast<float*>(y_user), s);
  else
    launch_permute_out(P.y_tree.get(), P.T.perm.get(), P.nT, static_cast<double*>(y_user), s);
}

void plan_zero_output(Plan& P, void* y_user, bool c64, hipStream_t s) {
  launch_zero_c128(P.y_tree.get(), P.nT, s);
  if (c64)
    launch_permute_out_c64(P.y_tree.get(), P.T.perm.get(), P.nT, static_cast<float*>(y_user), s);
  else
    launch_permute_out(P.y_tree.get(), P.T.perm.get(), P.nT, static_cast<double*>(y_user), s);
}

void plan_matvec(Plan& P, const void* v_user, void* y_user, bool c64, hipStream_t s,
                 bool use_static) {
  if (P.nT == 0) return;
  if (P.nS == 0) {  // no sources: y = 0
    plan_zero_output(P, y_user, c64, s);
    return;
  }
  if (use_static) {
    if (!P.sched_ready || !P.static_ready)
      fail(FDM_ERR_STATE, "the plan has no launch schedule for the static workspace");
  } else if (!P.sched_ready) {
    build_plan_schedule(P, s);
  }
  std::vector<M2LLaunch>& sched = use_static ? P.sched_static : P.sched;
  auto mark = [&](int i) {
    if (P.timing) FDM_HIP(hipEventRecord(P.ev[i], s));
  };
  const int p = P.levels;
  mark(0);
  if (c64)
    launch_permute_in_c64(static_cast<const float*>(v_user), P.S.perm.get(), P.nS,
                          P.v_tree.get(), s);
  else
    launch_permute_in(static_cast<const double*>(v_user), P.S.perm.get(), P.nS,
                      P.v_tree.get(), s);
  if (P.l_min <= p) launch_s2m(P, s);                   // forward transformation
  mark(1);
  if (P.l_min <= p)
    for (int l = p - 1; l >= P.l_min; --l) plan_m2m_level(P, l, s);
  mark(2);
  run_schedule(sched, P.heads.get(), P.prec, P.ip, P.tune, s,   // multiplication phase
               P.timing && P.launch_ev.size() == sched.size() ? P.launch_ev.data() : nullptr);
  mark(3);
  if (!p2p_queued(P, P.tune)) launch_p2p(P, s);         // near field (stored)
  mark(4);
  if (P.l_min <= p)
    for (int l = P.l_min; l < p; ++l) launch_l2l(P, l, s);  // backward transformation
  mark(5);
  launch_l2t(P, s);                                     // far field (added)
  mark(6);
  if (c64)
    launch_permute_out_c64(P.y_tree.get(), P.T.perm.get(), P.nT, static_cast<float*>(y_user), s);
  else
    launch_permute_out(P.y_tree.get(), P.T.perm.get(), P.nT, static_cast<double*>(y_user), s);
  mark(7);
  P.timed_run = P.timing;
  P.has_run = true;
}

}  // namespace fdm

// ====================================================================== C ABI
using namespace fdm;

namespace fdm {

void set_error(const std::string& m) { g_last_error = m; }
void clear_error() { g_last_error.clear(); }

void check_device_ptr(const void* p, const char* what) {
  if (!p) fail(FDM_ERR_INVALID_ARG, std::string(what) + " is NULL");
  hipPointerAttribute_t a{};
  if (hipPointerGetAttributes(&a, p) != hipSuccess) {
    (void)hipGetLastError();
    fail(FDM_ERR_INVALID_ARG, std::string(what) + " is not a device pointer");
  }
  if (a.type != hipMemoryTypeDevice && a.type != hipMemoryTypeManaged)
    fail(FDM_ERR_INVALID_ARG, std::string(what) + " is not device memory");
}

TuneConfig check_tune(const fdm_tune& t) {
  if (t.nb != 32 && t.nb != 64) fail(FDM_ERR_INVALID_ARG, "tune.nb must be 32 or 64");
  for (int v : {t.persistent, t.lpt, t.p2p_in_queue})
    if (v != 0 && v != 1) fail(FDM_ERR_INVALID_ARG, "tune flags must be 0 or 1");
  if (t.compact < 0 || t.compact > 2) fail(FDM_ERR_INVALID_ARG, "tune.compact must be 0, 1 or 2");
  TuneConfig c;
  c.nb = t.nb;
  c.persistent = t.persistent;
  c.lpt = t.lpt;
  c.p2p_in_queue = t.p2p_in_queue;
  c.compact = t.compact;
  return c;
}

fdm_tune to_c(const TuneConfig& c) {
  fdm_tune t{};
  t.nb = c.nb;
  t.persistent = c.persistent;
  t.lpt = c.lpt;
  t.p2p_in_queue = c.p2p_in_queue;
  t.compact = c.compact;
  return t;
}

void apply_plan_tune(Plan& P, const TuneConfig& c, hipStream_t s) {
  if (P.aca_kp && (c.nb != 64 || c.compact != 0 || c.p2p_in_queue != 0))
    fail(FDM_ERR_UNSUPPORTED,
         "low-rank couplings run 64 targets per item, no compaction, near field apart");
  const bool rebuild = c.nb != P.tune.nb;
  P.tune = c;
  if (rebuild && P.l_min <= P.levels) build_m2l_work(P, s);
  P.sched.clear();
  P.sched_static.clear();
  P.static_ready = false;
  P.sched_ready = false;
  FDM_HIP(hipStreamSynchronize(s));
}

}  // namespace fdm

extern "C" {

int fdm_build_tree_opts(const double* points_T, int64_t n_T, const double* points_S,
                        int64_t n_S, double kappa, const double box[6], int levels, int m,
                        const fdm_options* opts, void* stream, fdm_plan** out) {
  return guarded([&] {
    if (!out) fail(FDM_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (!opts) fail(FDM_ERR_INVALID_ARG, "opts is NULL");
    const int precision = opts->precision, l_hf = opts->l_hf;
    if (n_T < 0 || n_S < 0) fail(FDM_ERR_INVALID_ARG, "negative point count");
    if (n_T > INT32_MAX / 2 || n_S > INT32_MAX / 2)
      fail(FDM_ERR_UNSUPPORTED, "point count too large");
    if (!box) fail(FDM_ERR_INVALID_ARG, "box is NULL");
    if (!std::isfinite(kappa) || kappa < 0) fail(FDM_ERR_INVALID_ARG, "kappa must be finite and >= 0");
    if (levels < 0 || levels > 9) fail(FDM_ERR_INVALID_ARG, "levels must be in [0, 9]");
    if (m < 1 || m > 8) fail(FDM_ERR_INVALID_ARG, "m must be in [1, 8]");
    if (precision < FDM_PREC_FP64 || precision > FDM_PREC_BF16X6)
      fail(FDM_ERR_INVALID_ARG, "unknown precision");
    if (l_hf < -2 || l_hf > levels) fail(FDM_ERR_INVALID_ARG, "l_hf out of range");
    if (opts->bank_budget_bytes < 0) fail(FDM_ERR_INVALID_ARG, "negative bank budget");
    if (opts->full_bank != 0 && opts->full_bank != 1)
      fail(FDM_ERR_INVALID_ARG, "full_bank must be 0 or 1");
    if (!std::isfinite(opts->aca_eps) || opts->aca_eps < 0)
      fail(FDM_ERR_INVALID_ARG, "aca_eps must be finite and >= 0");
    if (opts->aca_rank != 0 && opts->aca_rank != 32 && opts->aca_rank != 64)
      fail(FDM_ERR_INVALID_ARG, "aca_rank must be 0, 32 or 64");
    if (opts->aca_chunk_bytes < 0) fail(FDM_ERR_INVALID_ARG, "negative aca_chunk_bytes");
    if (opts->aca_eps > 0 && precision != FDM_PREC_FP32)
      fail(FDM_ERR_UNSUPPORTED, "low-rank couplings run in the FP32 precision");
    if (opts->aca_eps > 0 && opts->bank_budget_bytes != 0)
      fail(FDM_ERR_INVALID_ARG, "low-rank couplings keep their bank resident");
    if (opts->n_max < 0) fail(FDM_ERR_INVALID_ARG, "negative n_max");
    TuneConfig tune;
    if (opts->tune.nb != 0)
      tune = check_tune(opts->tune);
    else if (precision == FDM_PREC_BF16X6)
      tune.nb = 32;  // its 64-target items run out of registers (see fdm.h)
    for (int d = 0; d < 3; ++d)
      if (!std::isfinite(box[d]) || !std::isfinite(box[d + 3]) || !(box[d + 3] > box[d]))
        fail(FDM_ERR_INVALID_ARG, "invalid box");
    const int K = (m + 1) * (m + 1) * (m + 1);
    if (opts->aca_eps > 0 && (K + 31) / 32 * 32 > kMaxKp)
      fail(FDM_ERR_UNSUPPORTED, "low-rank couplings need m <= 6");
    if (n_T) check_device_ptr(points_T, "points_T");
    if (n_S) check_device_ptr(points_S, "points_S");
    auto* h = new fdm_plan();
    try {
      Plan& P = h->p;
      P.nT = n_T;
      P.nS = n_S;
      P.kappa = kappa;
      for (int d = 0; d < 3; ++d) {
        P.lo[d] = box[d];
        P.hi[d] = box[d + 3];
      }
      P.levels = levels;
      P.m = m;
      P.prec = precision;
      P.l_hf = l_hf;
      P.tune = tune;
      P.bank_budget = opts->bank_budget_bytes;
      P.full_bank = opts->full_bank != 0;
      P.n_max = opts->n_max;
      if (opts->aca_eps > 0) {
        P.aca_eps = opts->aca_eps;
        P.aca_kp = opts->aca_rank ? opts->aca_rank : 64;
        if (opts->aca_chunk_bytes > 0) P.aca_T_budget = opts->aca_chunk_bytes;
        P.tune.nb = 64;
        P.tune.compact = 0;
        P.tune.p2p_in_queue = 0;
      }
      if (P.bank_budget > 0) {
        Interp ip{};
        ip.Kp = (K + 31) / 32 * 32;
        if (P.bank_budget < bank_matrix_bytes(precision, ip))
          fail(FDM_ERR_INVALID_ARG, "bank budget below one coupling matrix");
      }
      plan_build(P, points_T, points_S, static_cast<hipStream_t>(stream));
    } catch (...) {
      (void)hipStreamSynchronize(static_cast<hipStream_t>(stream));
      delete h;
      throw;
    }
    *out = h;
  });
}

int fdm_build_tree_ex(const double* points_T, int64_t n_T, const double* points_S,
                      int64_t n_S, double kappa, const double box[6], int levels, int m,
                      int precision, int l_hf, void* stream, fdm_plan** out) {
  fdm_options o{};
  o.precision = precision;
  o.l_hf = l_hf;
  return fdm_build_tree_opts(points_T, n_T, points_S, n_S, kappa, box, levels, m, &o, stream,
                             out);
}

int fdm_build_tree(const double* points_T, int64_t n_T, const double* points_S,
                   int64_t n_S, double kappa, const double box[6], int levels, int m,
                   int precision, void* stream, fdm_plan** out) {
  return fdm_build_tree_ex(points_T, n_T, points_S, n_S, kappa, box, levels, m, precision,
                           -2, stream, out);
}

int fdm_plan_get_tune(const fdm_plan* plan, fdm_tune* out) {
  return guarded([&] {
    if (!plan || !out) fail(FDM_ERR_INVALID_ARG, "NULL argument");
    *out = to_c(plan->p.tune);
  });
}

int fdm_plan_set_tune(fdm_plan* plan, const fdm_tune* tune, void* stream) {
  return guarded([&] {
    if (!plan || !tune) fail(FDM_ERR_INVALID_ARG, "NULL argument");
    Plan& P = plan->p;
    if (P.batch_owner) fail(FDM_ERR_STATE, "the plan belongs to a batch");
    apply_plan_tune(P, check_tune(*tune), static_cast<hipStream_t>(stream));
  });
}

static int matvec_entry(fdm_plan* plan, const void* v, void* y, void* stream, bool c64) {
  return guarded([&] {
    if (!plan) fail(FDM_ERR_INVALID_ARG, "plan is NULL");
    Plan& P = plan->p;
    if (P.nS) check_device_ptr(v, "v");
    if (P.nT) check_device_ptr(y, "y");
    const int64_t w = c64 ? 8 : 16;
    if (P.nS && P.nT) {
      const char* a = static_cast<const char*>(v);
      const char* b = static_cast<const char*>(y);
      if (a < b + w * P.nT && b < a + w * P.nS) fail(FDM_ERR_INVALID_ARG, "v and y overlap");
    }
    plan_matvec(P, v, y, c64, static_cast<hipStream_t>(stream));
  });
}

int fdm_plan_matvec(fdm_plan* plan, const void* v, void* y, void* stream) {
  return matvec_entry(plan, v, y, stream, false);
}

int fdm_plan_matvec_c64(fdm_plan* plan, const void* v, void* y, void* stream) {
  return matvec_entry(plan, v, y, stream, true);
}

int fdm_plan_set_timing(fdm_plan* plan, int enable) {
  return guarded([&] {
    if (!plan) fail(FDM_ERR_INVALID_ARG, "plan is NULL");
    Plan& P = plan->p;
    if (enable && !P.timing) {
      for (auto& e : P.ev) FDM_HIP(hipEventCreate(&e));
    } else if (!enable && P.timing) {
      FDM_HIP(hipDeviceSynchronize());
      for (auto& e : P.ev) {
        (void)hipEventDestroy(e);
        e = nullptr;
      }
    }
    P.timing = enable != 0;
    P.timed_run = false;
    if (P.sched_ready) plan_launch_events(P);
  });
}

int fdm_plan_prepare(fdm_plan* plan, void* stream) {
  return guarded([&] {
    if (!plan) fail(FDM_ERR_INVALID_ARG, "plan is NULL");
    Plan& P = plan->p;
    if (!P.sched_ready) build_plan_schedule(P, static_cast<hipStream_t>(stream));
  });
}

int fdm_plan_coupling_launches(const fdm_plan* plan, int* n) {
  return guarded([&] {
    if (!plan || !n) fail(FDM_ERR_INVALID_ARG, "NULL argument");
    if (!plan->p.sched_ready) fail(FDM_ERR_STATE, "the plan has no launch schedule yet");
    *n = static_cast<int>(plan->p.sched.size());
  });
}

int fdm_plan_wait_launch(const fdm_plan* plan, int i, double* ms) {
  return guarded([&] {
    if (!plan || !ms) fail(FDM_ERR_INVALID_ARG, "NULL argument");
    const Plan& P = plan->p;
    if (!P.timing || !P.timed_run) fail(FDM_ERR_STATE, "no timed matvec");
    if (i < 0 || i >= static_cast<int>(P.launch_ev.size()))
      fail(FDM_ERR_INVALID_ARG, "launch index out of range");
    FDM_HIP(hipEventSynchronize(P.launch_ev[i]));
    float t = 0;
    FDM_HIP(hipEventElapsedTime(&t, P.ev[0], P.launch_ev[i]));
    *ms = t;
  });
}

int fdm_plan_phase_ms(const fdm_plan* plan, double ms[7]) {
  return guarded([&] {
    if (!plan || !ms) fail(FDM_ERR_INVALID_ARG, "NULL argument");
    const Plan& P = plan->p;
    if (!P.timing || !P.timed_run) fail(FDM_ERR_STATE, "no timed matvec");
    FDM_HIP(hipEventSynchronize(P.ev[7]));
    // S2M, M2M, M2L (with the near field when it shares the launch), L2L,
    // L2T, near field
    const int pairs[6][2] = {{0, 1}, {1, 2}, {2, 3}, {4, 5}, {5, 6}, {3, 4}};
    for (int i = 0; i < 6; ++i) {
      float t = 0;
      FDM_HIP(hipEventElapsedTime(&t, P.ev[pairs[i][0]], P.ev[pairs[i][1]]));
      ms[i] = t;
    }
    float t = 0;
    FDM_HIP(hipEventElapsedTime(&t, P.ev[0], P.ev[7]));
    ms[6] = t;
  });
}

int fdm_plan_destroy(fdm_plan* plan) {
  return guarded([&] {
    if (!plan) return;
    if (plan->p.batch_owner) fail(FDM_ERR_STATE, "the plan belongs to a batch");
    (void)hipDeviceSynchronize();
    for (auto& e : plan->p.ev)
      if (e) (void)hipEventDestroy(e);
    for (auto& e : plan->p.launch_ev)
      if (e) (void)hipEventDestroy(e);
    delete plan;
  });
}

int fdm_plan_stats(const fdm_plan* plan, fdm_stats* out) {
  return guarded([&] {
    if (!plan || !out) fail(FDM_ERR_INVALID_ARG, "NULL argument");
    const Plan& P = plan->p;
    fdm_stats st{};
    st.n_T = P.nT;
    st.n_S = P.nS;
    st.levels = P.levels;
    st.m = P.m;
    st.K = P.ip.K;
    st.precision = P.prec;
    st.l_hf = P.l_hf;
    st.l_min = P.l_min;
    st.n_couplings = P.n_couplings;
    st.n_stored_couplings = P.n_stored;
    st.n_bank_matrices = P.bank_budget == 0 ? P.n_bank_stored : P.n_bank;
    st.aca_rank_cap = P.aca_kp;
    st.aca_rank_max = 0;
    st.aca_rank_mean = 0.0;
    for (int32_t r : P.aca_rank) {
      st.aca_rank_max = std::max(st.aca_rank_max, r);
      st.aca_rank_mean += r;
    }
    if (!P.aca_rank.empty()) st.aca_rank_mean /= static_cast<double>(P.aca_rank.size());
    st.aca_flops = 0.0;
    for (size_t b = 0; b < P.aca_rank.size() && b < P.bank_work.size(); ++b)
      st.aca_flops += 16.0 * P.ip.K * P.aca_rank[b] * static_cast<double>(P.bank_work[b]);
    st.aca_issued_flops = 16.0 * P.ip.Kp * P.aca_issued_cols;
    st.near_pairs = P.near_pairs;
    st.near_entries = P.near_entries;
    st.m2l_columns = issued_columns(P, P.tune);
    st.device_bytes = P.tally;
    st.setup_ms = P.setup_ms;
    *out = st;
  });
}

int fdm_dense_matvec(const double* points_T, int64_t n_T, const double* points_S,
                     int64_t n_S, double kappa, const void* v, void* y, void* stream) {
  return guarded([&] {
    if (n_T < 0 || n_S < 0) fail(FDM_ERR_INVALID_ARG, "negative point count");
    if (!std::isfinite(kappa) || kappa < 0) fail(FDM_ERR_INVALID_ARG, "kappa must be finite and >= 0");
    if (n_T == 0) return;
    check_device_ptr(points_T, "points_T");
    check_device_ptr(y, "y");
    if (n_S) {
      check_device_ptr(points_S, "points_S");
      check_device_ptr(v, "v");
    }
    launch_dense(points_T, n_T, points_S, n_S, kappa, static_cast<const double*>(v),
                 static_cast<double*>(y), static_cast<hipStream_t>(stream));
  });
}

const char* fdm_last_error(void) { return g_last_error.c_str(); }

const char* fdm_version(void) { return "fdm-gfx950 0.1"; }

}  // extern "C"
