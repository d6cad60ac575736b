// Batched matvecs over many plans from one device queue, HIP-graph capture
// of the whole batched matvec, and the launch-shape autotuner (C ABI).
#include <algorithm>
#include <set>

#include "plan.hpp"
#include "capi.hpp"

namespace fdm {

namespace {

void invalidate_graph(fdm_batch& b) {
  if (b.graph) (void)hipGraphExecDestroy(b.graph);
  b.graph = nullptr;
  b.graph_v.clear();
  b.graph_y.clear();
  b.graph_stream = nullptr;
  b.graph_c64 = -1;
}

void batch_schedule(fdm_batch& b, hipStream_t s) {
  invalidate_graph(b);
  if (b.aca_kp) {  // low-rank couplings: launch pairs over every plan's groups
    b.sched = build_aca_schedule(b.plans, b.tune, b.aca_T, int64_t(8) << 30, &b.tally, s);
    b.heads.alloc(std::max<size_t>(b.sched.size(), 1), &b.tally);
    return;
  }
  const int64_t mb = bank_matrix_bytes(b.prec, b.ip);
  const int64_t ws_mats = b.ws.size() / mb;
  b.sched = build_schedule(b.plans, b.tune, b.ws.get(), ws_mats, s);
  b.heads.alloc(std::max<size_t>(b.sched.size(), 1), &b.tally);
}

// Every launch of one batched matvec, enqueued on s.
void batch_enqueue(fdm_batch& b, const void* const* v, void* const* y, bool c64,
                   hipStream_t s) {
  for (size_t i = 0; i < b.plans.size(); ++i) {
    Plan& P = *b.plans[i];
    if (P.nT > 0 && P.nS > 0) plan_upward(P, v[i], c64, s);
  }
  run_schedule(b.sched, b.heads.get(), b.prec, b.ip, b.tune, s);
  for (size_t i = 0; i < b.plans.size(); ++i) {
    Plan& P = *b.plans[i];
    if (P.nT == 0) continue;
    if (P.nS == 0) {
      plan_zero_output(P, y[i], c64, s);
      continue;
    }
    if (!p2p_queued(P, b.tune)) launch_p2p(P, s);
    plan_downward(P, y[i], c64, s);
  }
}

void batch_run(fdm_batch& b, const void* const* v, void* const* y, bool c64, hipStream_t s) {
  const size_t n = b.plans.size();
  if (!b.use_graph || s == nullptr) {
    batch_enqueue(b, v, y, c64, s);
    return;
  }
  const bool same = b.graph && b.graph_stream == s && b.graph_c64 == int(c64) &&
                    std::equal(v, v + n, b.graph_v.begin()) &&
                    std::equal(y, y + n, b.graph_y.begin());
  if (!same) {
    invalidate_graph(b);
    FDM_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    try {
      batch_enqueue(b, v, y, c64, s);
    } catch (...) {
      hipGraph_t junk = nullptr;
      (void)hipStreamEndCapture(s, &junk);
      if (junk) (void)hipGraphDestroy(junk);
      throw;
    }
    hipGraph_t g = nullptr;
    FDM_HIP(hipStreamEndCapture(s, &g));
    hipGraphExec_t ex = nullptr;
    const hipError_t e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    FDM_HIP(e);
    b.graph = ex;
    b.graph_v.assign(v, v + n);
    b.graph_y.assign(y, y + n);
    b.graph_stream = s;
    b.graph_c64 = int(c64);
  }
  FDM_HIP(hipGraphLaunch(b.graph, s));
}

void check_vectors(const fdm_batch& b, const void* const* v, void* const* y, int c64) {
  if (!v || !y) fail(FDM_ERR_INVALID_ARG, "v or y is NULL");
  const int64_t w = c64 ? 8 : 16;
  for (size_t i = 0; i < b.plans.size(); ++i) {
    const Plan& P = *b.plans[i];
    if (P.nS) check_device_ptr(v[i], "v[i]");
    if (P.nT) check_device_ptr(y[i], "y[i]");
    if (P.nS && P.nT) {
      const char* a = static_cast<const char*>(v[i]);
      const char* c = static_cast<const char*>(y[i]);
      if (a < c + w * P.nT && c < a + w * P.nS) fail(FDM_ERR_INVALID_ARG, "v[i] and y[i] overlap");
    }
  }
}

// Elapsed milliseconds of f() enqueued on s.
template <class F>
double time_on_stream(hipStream_t s, F&& f) {
  hipEvent_t e0 = nullptr, e1 = nullptr;
  FDM_HIP(hipEventCreate(&e0));
  FDM_HIP(hipEventCreate(&e1));
  float ms = 0;
  try {
    FDM_HIP(hipEventRecord(e0, s));
    f();
    FDM_HIP(hipEventRecord(e1, s));
    FDM_HIP(hipEventSynchronize(e1));
    FDM_HIP(hipEventElapsedTime(&ms, e0, e1));
  } catch (...) {
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    throw;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return ms;
}

// Launch shapes: nb x persistent x lpt with the near field and compaction
// as set; then, where the precision has compacted items (compactable), the
// other two compaction modes at (64, persistent, heaviest first).
std::vector<TuneConfig> candidates(bool persistent_only, int p2p_in_queue, int compact,
                                   bool compactable) {
  std::vector<TuneConfig> out;
  for (int nb : {64, 32})
    for (int pers : {1, 0}) {
      if (persistent_only && !pers) continue;
      for (int lpt : {1, 0}) {
        TuneConfig c;
        c.nb = nb;
        c.persistent = pers;
        c.lpt = lpt;
        c.p2p_in_queue = p2p_in_queue;
        c.compact = compact;
        out.push_back(c);
      }
    }
  if (compactable)
    for (int mode : {0, 1, 2}) {
      if (mode == compact) continue;
      TuneConfig c;
      c.nb = 64;
      c.persistent = 1;
      c.lpt = 1;
      c.p2p_in_queue = p2p_in_queue;
      c.compact = mode;
      out.push_back(c);
    }
  return out;
}

}  // namespace

}  // namespace fdm

using namespace fdm;

extern "C" {

int fdm_plan_autotune(fdm_plan* plan, const void* v, void* y, int c64, int max_candidates,
                      void* stream, fdm_tune* best, double* ms) {
  return guarded([&] {
    if (!plan) fail(FDM_ERR_INVALID_ARG, "plan is NULL");
    Plan& P = plan->p;
    if (P.batch_owner) fail(FDM_ERR_STATE, "the plan belongs to a batch");
    const auto cand = candidates(false, P.tune.p2p_in_queue, P.tune.compact,
                                 compact_supported(P.prec, 64) && !P.aca_kp);
    if (max_candidates < 1 || max_candidates > static_cast<int>(cand.size()))
      fail(FDM_ERR_INVALID_ARG, "max_candidates out of range");
    if (P.nS) check_device_ptr(v, "v");
    if (P.nT) check_device_ptr(y, "y");
    hipStream_t s = static_cast<hipStream_t>(stream);
    plan_matvec(P, v, y, c64 != 0, s);  // the result, and moments to time on
    FDM_HIP(hipStreamSynchronize(s));
    double best_ms = -1;
    TuneConfig keep = P.tune;
    for (int i = 0; i < max_candidates; ++i) {
      if (P.aca_kp && cand[i].nb != 64) {  // low-rank items hold 64 targets
        if (ms) ms[i] = -1.0;
        continue;
      }
      apply_plan_tune(P, cand[i], s);
      build_plan_schedule(P, s);
      const double t = time_on_stream(s, [&] {
        run_schedule(P.sched, P.heads.get(), P.prec, P.ip, P.tune, s);
      });
      if (ms) ms[i] = t;
      if (best_ms < 0 || t < best_ms) {
        best_ms = t;
        keep = cand[i];
      }
    }
    apply_plan_tune(P, keep, s);
    if (best) *best = to_c(keep);
  });
}

int fdm_batch_create(fdm_plan* const* plans, int n, int64_t workspace_bytes, void* stream,
                     fdm_batch** out) {
  return guarded([&] {
    if (!out) fail(FDM_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (!plans || n < 1) fail(FDM_ERR_INVALID_ARG, "no plans");
    if (workspace_bytes < 0) fail(FDM_ERR_INVALID_ARG, "negative workspace size");
    std::set<const fdm_plan*> seen;
    for (int i = 0; i < n; ++i) {
      if (!plans[i]) fail(FDM_ERR_INVALID_ARG, "NULL plan");
      if (!seen.insert(plans[i]).second) fail(FDM_ERR_INVALID_ARG, "a plan appears twice");
      if (plans[i]->p.batch_owner) fail(FDM_ERR_STATE, "a plan already belongs to a batch");
      if (plans[i]->p.m != plans[0]->p.m || plans[i]->p.prec != plans[0]->p.prec)
        fail(FDM_ERR_UNSUPPORTED, "plans of a batch must share m and precision");
      if (plans[i]->p.aca_kp != plans[0]->p.aca_kp)
        fail(FDM_ERR_UNSUPPORTED,
             "plans of a batch must all have low-rank couplings with one rank cap, or none");
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    auto* b = new fdm_batch();
    try {
      b->prec = plans[0]->p.prec;
      b->ip = plans[0]->p.ip;
      b->tune.nb = plans[0]->p.tune.nb;
      b->tune.persistent = 1;
      b->tune.lpt = 1;
      b->tune.p2p_in_queue = 1;
      b->tune.compact = plans[0]->p.tune.compact;
      b->aca_kp = plans[0]->p.aca_kp;
      if (b->aca_kp) {  // low-rank items: 64 targets, no compaction, near field apart
        b->tune.p2p_in_queue = 0;
        b->tune.compact = 0;
      }
      const int64_t mb = bank_matrix_bytes(b->prec, b->ip);
      int64_t need = 0;
      for (int i = 0; i < n; ++i) {
        Plan& P = plans[i]->p;
        if (P.tune.nb != b->tune.nb) {
          TuneConfig c = P.tune;
          c.nb = b->tune.nb;
          apply_plan_tune(P, c, s);
        }
        if (P.bank_budget > 0 && !P.base_items.empty()) need += P.n_bank * mb;
        b->plans.push_back(&P);
      }
      if (need > 0) {
        int64_t ws = workspace_bytes;
        if (ws == 0) {
          size_t free_b = 0, total_b = 0;
          FDM_HIP(hipMemGetInfo(&free_b, &total_b));
          ws = std::min<int64_t>(need, static_cast<int64_t>(free_b / 2));
        }
        ws = std::min(ws, need) / mb * mb;
        if (ws < mb) fail(FDM_ERR_OUT_OF_MEMORY, "workspace below one coupling matrix");
        b->ws.alloc(ws, &b->tally);
      }
      batch_schedule(*b, s);
      for (Plan* P : b->plans) P->batch_owner = b;
    } catch (...) {
      (void)hipStreamSynchronize(s);
      delete b;
      throw;
    }
    *out = b;
  });
}

int fdm_batch_matvec(fdm_batch* batch, const void* const* v, void* const* y, int c64,
                     void* stream) {
  return guarded([&] {
    if (!batch) fail(FDM_ERR_INVALID_ARG, "batch is NULL");
    check_vectors(*batch, v, y, c64);
    batch_run(*batch, v, y, c64 != 0, static_cast<hipStream_t>(stream));
  });
}

int fdm_batch_set_graph(fdm_batch* batch, int enable) {
  return guarded([&] {
    if (!batch) fail(FDM_ERR_INVALID_ARG, "batch is NULL");
    batch->use_graph = enable != 0;
    if (!batch->use_graph) invalidate_graph(*batch);
  });
}

int fdm_batch_get_tune(const fdm_batch* batch, fdm_tune* out) {
  return guarded([&] {
    if (!batch || !out) fail(FDM_ERR_INVALID_ARG, "NULL argument");
    *out = to_c(batch->tune);
  });
}

int fdm_batch_set_tune(fdm_batch* batch, const fdm_tune* tune, void* stream) {
  return guarded([&] {
    if (!batch || !tune) fail(FDM_ERR_INVALID_ARG, "NULL argument");
    const TuneConfig c = check_tune(*tune);
    hipStream_t s = static_cast<hipStream_t>(stream);
    FDM_HIP(hipStreamSynchronize(s));
    for (Plan* P : batch->plans)
      if (P->tune.nb != c.nb) {
        TuneConfig pc = P->tune;
        pc.nb = c.nb;
        apply_plan_tune(*P, pc, s);
      }
    batch->tune = c;
    batch_schedule(*batch, s);
  });
}

int fdm_batch_autotune(fdm_batch* batch, const void* const* v, void* const* y, int c64,
                       int max_candidates, void* stream, fdm_tune* best, double* ms) {
  return guarded([&] {
    if (!batch) fail(FDM_ERR_INVALID_ARG, "batch is NULL");
    fdm_batch& b = *batch;
    const auto cand = candidates(true, b.aca_kp ? 0 : 1, b.tune.compact,
                                 compact_supported(b.prec, 64) && !b.aca_kp);
    if (max_candidates < 1 || max_candidates > static_cast<int>(cand.size()))
      fail(FDM_ERR_INVALID_ARG, "max_candidates out of range");
    check_vectors(b, v, y, c64);
    hipStream_t s = static_cast<hipStream_t>(stream);
    batch_enqueue(b, v, y, c64 != 0, s);  // the result, and moments to time on
    FDM_HIP(hipStreamSynchronize(s));
    double best_ms = -1;
    TuneConfig keep = b.tune;
    auto apply = [&](const TuneConfig& c) {
      for (Plan* P : b.plans)
        if (P->tune.nb != c.nb) {
          TuneConfig pc = P->tune;
          pc.nb = c.nb;
          apply_plan_tune(*P, pc, s);
        }
      b.tune = c;
      batch_schedule(b, s);
    };
    for (int i = 0; i < max_candidates; ++i) {
      if (b.aca_kp && (cand[i].nb != 64 || cand[i].p2p_in_queue || cand[i].compact)) {
        if (ms) ms[i] = -1.0;  // low-rank items: 64 targets, no compaction, near field apart
        continue;
      }
      apply(cand[i]);
      const double t = time_on_stream(s, [&] {
        run_schedule(b.sched, b.heads.get(), b.prec, b.ip, b.tune, s);
      });
      if (ms) ms[i] = t;
      if (best_ms < 0 || t < best_ms) {
        best_ms = t;
        keep = cand[i];
      }
    }
    apply(keep);
    if (best) *best = to_c(keep);
  });
}

int fdm_batch_destroy(fdm_batch* batch) {
  return guarded([&] {
    if (!batch) return;
    (void)hipDeviceSynchronize();
    invalidate_graph(*batch);
    for (Plan* P : batch->plans) P->batch_owner = nullptr;
    delete batch;
  });
}

}  // extern "C"
