// Host side of the coupling step (Sect. 2.6, M2L): the coupling bank, the
// work items of a plan, and the launch schedules that run them -- for one
// plan or for a batch of plans, with resident banks or with banks generated
// into a bounded workspace a range of matrices at a time.
#include <algorithm>
#include <map>

#include "plan.hpp"

namespace fdm {

int64_t bank_matrix_bytes(int prec, const Interp& ip) {
  const int64_t per = int64_t(ip.Kp) * ip.Kp;
  if (prec == FDM_PREC_FP64) return 2 * per * 8;
  if (prec == FDM_PREC_BF16X3) return 4 * per * 2;
  if (prec == FDM_PREC_BF16X6) return 6 * per * 2;
  return 2 * per * 4;
}

namespace {

BankLevel bank_level(const Plan& P, int l) {
  const LevelData& Ld = P.L[l];
  return BankLevel{Ld.dirvec.get(), {Ld.h[0], Ld.h[1], Ld.h[2]}, P.kappa, l, Ld.nd};
}

// Whether base item i runs with compacted columns under `cfg`: mode 1 when
// its compacted tiles (32 columns each) save at least a fifth of the plain
// item's columns (nb per offset) -- items at sparse levels and at the
// domain boundary.
bool item_compact(const Plan& P, size_t i, const TuneConfig& cfg) {
  if (!cfg.compact || !compact_supported(P.prec, cfg.nb) || P.tune.nb != cfg.nb) return false;
  if (cfg.compact == 2) return true;
  return 5 * 32 * int64_t(P.item_tiles[i]) <= 4 * int64_t(cfg.nb) * P.base_items[i].vo_count;
}

}  // namespace

int64_t issued_columns(const Plan& P, const TuneConfig& cfg) {
  int64_t n = 0;
  for (size_t i = 0; i < P.base_items.size(); ++i)
    n += item_compact(P, i, cfg) ? 32 * int64_t(P.item_tiles[i])
                                 : int64_t(P.tune.nb) * P.base_items[i].vo_count;
  return n;
}

namespace {

// `bank` holds bank id bank_id0 as its first matrix.
M2LDesc level_desc(const Plan& P, int l, const void* bank, int64_t bank_id0) {
  const LevelData& Ld = P.L[l];
  M2LDesc d{};
  d.gridS = P.adaptive() ? P.gridS_alive[l].get() : P.S.grid[l].get();
  d.keyT = P.T.key[l].get();
  d.mom = P.prec == FDM_PREC_FP64    ? static_cast<const void*>(Ld.mom64.get())
          : P.prec == FDM_PREC_BF16X6 ? static_cast<const void*>(Ld.mom16.get())
                                      : static_cast<const void*>(Ld.mom32.get());
  d.out = Ld.loc64.get();  // FP64 coupling result, completed in place by L2L
  d.tgt_list = P.tgt_list.get();
  d.valid_off = P.valid_off.get();
  d.offtab = P.offtab.get();
  const int64_t mb = bank_matrix_bytes(P.prec, P.ip);
  d.bank = reinterpret_cast<const void*>(reinterpret_cast<uintptr_t>(bank) -
                                         static_cast<uintptr_t>(bank_id0 * mb));
  d.nd = Ld.nd;
  d.level = l;
  d.K = P.ip.K;
  d.kp = P.aca_kp;
  d.rows = P.ip.Kp;
  return d;
}

// Descriptor of row block rb of a level whose matrices are split into row
// blocks of `block` rows: bank and out point at the block's first row (row
// r of a matrix sits at offset r in every layout: k-major planes, and the
// BF16 fragments, 512 values per 32 rows of a slab; the FP64 result has
// stride Kp per (target, direction)).
M2LDesc row_block_desc(const Plan& P, M2LDesc d, int rb, int block) {
  const int64_t r0 = int64_t(rb) * block;
  const int64_t elem = P.prec == FDM_PREC_FP64 ? 8 : P.prec == FDM_PREC_FP32 ? 4 : 2;
  const int64_t shift = (P.prec == FDM_PREC_BF16X3 || P.prec == FDM_PREC_BF16X6) ? r0 * 16 : r0;
  d.bank = reinterpret_cast<const void*>(reinterpret_cast<uintptr_t>(d.bank) +
                                         static_cast<uintptr_t>(shift * elem));
  d.out = static_cast<double2*>(d.out) + r0;
  d.rows = static_cast<int32_t>(std::min<int64_t>(block, P.ip.Kp - r0));
  return d;
}

const void* resident_bank(const Plan& P) {
  if (P.aca_kp) return P.aca_bank.get();
  if (P.prec == FDM_PREC_FP64) return P.bank64.get();
  if (P.prec == FDM_PREC_BF16X3 || P.prec == FDM_PREC_BF16X6) return P.bank16.get();
  return P.bank32.get();
}

// Host image of one launch while a schedule is assembled.
struct LaunchBuilder {
  std::vector<M2LItem> items, p2p_items;
  std::vector<double> weight;  // per coupling item: MFMA column tiles it issues
  std::vector<M2LDesc> descs;
  std::vector<P2PDesc> p2p;
  std::vector<int32_t> gen_info;
  std::vector<BankLevel> gen_levels;
  std::map<std::pair<const Plan*, int>, int32_t> gen_level_index;
  int64_t n_gen = 0;
};

// Items of plan P restricted to the bank ids [b0, b1), whose matrices sit
// at `bank` with bank id b0 at position slot0.
void add_source(LaunchBuilder& B, const Plan& P, int64_t b0, int64_t b1, const void* bank,
                int64_t slot0, const TuneConfig& cfg, std::vector<uint8_t>& emitted) {
  // one descriptor per level, or per (level, row block) for matrices with
  // more rows than a workgroup covers
  const int row_blocks = m2l_row_blocks(P.ip.Kp);
  const int block = m2l_threads(P.ip.Kp) / 2;  // rows per block (one wave per 32)
  std::vector<int32_t> desc_of(P.levels + 1, -1);
  for (int l = std::max(P.l_min, 0); l <= P.levels; ++l) {
    desc_of[l] = static_cast<int32_t>(B.descs.size());
    const M2LDesc d = level_desc(P, l, bank, b0 - slot0);
    if (row_blocks == 1)
      B.descs.push_back(d);
    else
      for (int rb = 0; rb < row_blocks; ++rb) B.descs.push_back(row_block_desc(P, d, rb, block));
  }
  const auto& vo = P.valid_off_h;
  for (size_t i = 0; i < P.base_items.size(); ++i) {
    const M2LItem& it = P.base_items[i];
    M2LItem o = it;
    o.desc = desc_of[it.desc];
    o.compact = item_compact(P, i, cfg) ? 1 : 0;
    if (it.vo_count == 0) {  // no source box: stored as zero once
      if (emitted[i]) continue;
      o.first = 1;
    } else {
      const auto first = vo.begin() + it.vo_begin, last = first + it.vo_count;
      const auto lo = std::lower_bound(first, last, static_cast<int32_t>(b0));
      const auto hi = std::lower_bound(lo, last, b1 > INT32_MAX ? INT32_MAX : static_cast<int32_t>(b1));
      if (lo == hi) continue;
      o.vo_begin = static_cast<int32_t>(lo - vo.begin());
      o.vo_count = static_cast<int32_t>(hi - lo);
      o.first = emitted[i] ? 0 : 1;
    }
    emitted[i] = 1;
    // one item per row block of the matrices (disjoint rows of the result)
    for (int rb = 0; rb < row_blocks; ++rb) {
      M2LItem r = o;
      r.desc = o.desc + rb;
      B.items.push_back(r);
      // plain: nb / 32 tiles per offset; compacted: the item's tiles, shared
      // over its parts in proportion to their offsets
      B.weight.push_back(o.compact ? double(P.item_tiles[i]) * o.vo_count /
                                         std::max(it.vo_count, 1)
                                   : double(o.vo_count) * cfg.nb / 32);
    }
  }
}

void add_generation(LaunchBuilder& B, const Plan& P, int64_t b0, int64_t b1) {
  for (int64_t b = b0; b < b1; ++b) {
    const int32_t* in = &P.bank_info[5 * b];
    const auto key = std::make_pair(&P, static_cast<int>(in[0]));
    auto f = B.gen_level_index.find(key);
    int32_t li;
    if (f == B.gen_level_index.end()) {
      li = static_cast<int32_t>(B.gen_levels.size());
      B.gen_levels.push_back(bank_level(P, in[0]));
      B.gen_level_index[key] = li;
    } else {
      li = f->second;
    }
    B.gen_info.insert(B.gen_info.end(), {li, in[1], in[2], in[3], in[4]});
    ++B.n_gen;
  }
}

void add_near_field(LaunchBuilder& B, Plan& P, int chunk) {
  if (P.nT == 0 || P.nS == 0 || P.adaptive()) return;  // adaptive: own launch
  const int32_t d = static_cast<int32_t>(B.p2p.size());
  B.p2p.push_back(p2p_desc(P));
  for (int64_t j = 0; j < P.nT; j += chunk) {
    const int n = static_cast<int>(std::min<int64_t>(chunk, P.nT - j));
    B.p2p_items.push_back(M2LItem{-d - 1, 0, static_cast<int32_t>(j), n, 0, 0, 1, 0});
  }
}

M2LLaunch upload(LaunchBuilder& B, const TuneConfig& cfg, int prec, int Kp, void* ws,
                 hipStream_t s) {
  if (cfg.lpt) {  // heaviest items first (longest-processing-time order)
    std::vector<size_t> order(B.items.size());
    for (size_t i = 0; i < order.size(); ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(),
                     [&](size_t a, size_t b) { return B.weight[a] > B.weight[b]; });
    std::vector<M2LItem> sorted(order.size());
    for (size_t i = 0; i < order.size(); ++i) sorted[i] = B.items[order[i]];
    B.items.swap(sorted);
  }
  M2LLaunch L;
  L.n_items = static_cast<int64_t>(B.items.size() + B.p2p_items.size());
  L.n_p2p_items = static_cast<int64_t>(B.p2p_items.size());
  for (const M2LItem& it : B.items) L.has_parts |= (it.first & 1) == 0;
  L.resident_wgs = m2l_resident_groups(prec, cfg.nb, Kp, L.has_parts);
  B.items.insert(B.items.end(), B.p2p_items.begin(), B.p2p_items.end());
  to_device(L.items, B.items, s, nullptr);
  to_device(L.descs, B.descs, s, nullptr);
  to_device(L.p2p, B.p2p, s, nullptr);
  L.n_gen = B.n_gen;
  if (B.n_gen) {
    to_device(L.gen_info, B.gen_info, s, nullptr);
    to_device(L.gen_levels, B.gen_levels, s, nullptr);
    L.gen_dst = ws;
  }
  FDM_HIP(hipStreamSynchronize(s));  // host images go out of scope
  return L;
}

}  // namespace

std::vector<M2LLaunch> build_schedule(const std::vector<Plan*>& plans, const TuneConfig& cfg,
                                      void* ws, int64_t ws_matrices, hipStream_t s) {
  std::vector<LaunchBuilder> B;
  std::vector<std::vector<uint8_t>> emitted(plans.size());
  for (size_t p = 0; p < plans.size(); ++p) emitted[p].assign(plans[p]->base_items.size(), 0);
  // resident banks: one launch
  for (size_t p = 0; p < plans.size(); ++p) {
    Plan& P = *plans[p];
    if (P.base_items.empty() || P.bank_budget != 0) continue;
    if (B.empty()) B.emplace_back();
    add_source(B[0], P, 0, P.n_bank, resident_bank(P), 0, cfg, emitted[p]);
  }
  // streamed banks: consecutive bank ids packed into launches of at most
  // ws_matrices matrices, and of about equal work (blocks using the
  // matrices): as few launches as the workspace allows, none much longer
  // than the others (the leaf levels have few matrices but most blocks)
  int64_t n_mats = 0;
  double total_work = 0;
  for (Plan* P : plans) {
    if (P->base_items.empty() || P->bank_budget == 0) continue;
    n_mats += P->n_bank;
    for (int64_t w : P->bank_work) total_work += static_cast<double>(w);
  }
  const int64_t n_min = ws_matrices > 0 ? (n_mats + ws_matrices - 1) / ws_matrices : 0;
  const double target = n_min > 0 ? total_work / static_cast<double>(n_min) : 0.0;
  int64_t left = 0;
  double acc = 0;
  for (size_t p = 0; p < plans.size(); ++p) {
    Plan& P = *plans[p];
    if (P.base_items.empty() || P.bank_budget == 0) continue;
    if (ws_matrices <= 0) fail(FDM_ERR_INVALID_ARG, "no workspace for a streamed bank");
    for (int64_t b = 0; b < P.n_bank;) {
      if (left == 0) {
        if (B.empty() || B.back().n_gen > 0 || !B.back().items.empty()) B.emplace_back();
        left = ws_matrices;
        acc = 0;
      }
      int64_t e = b;
      while (e < P.n_bank && e - b < left) {
        const double w = static_cast<double>(P.bank_work[e]);
        if (acc > 0 && acc + w > target) break;
        acc += w;
        ++e;
      }
      if (e == b) {  // this launch's work is full: next launch
        left = 0;
        continue;
      }
      const int64_t slot0 = ws_matrices - left;
      add_generation(B.back(), P, b, e);
      add_source(B.back(), P, b, e, ws, slot0, cfg, emitted[p]);
      left -= e - b;
      if (e < P.n_bank) left = 0;  // full (matrices or work): next launch
      b = e;
    }
  }
  if (cfg.p2p_in_queue && !plans.empty() &&
      p2p_queue_supported(plans[0]->prec, plans[0]->ip.Kp)) {
    if (B.empty()) B.emplace_back();
    for (Plan* P : plans) add_near_field(B.back(), *P, m2l_threads(P->ip.Kp));
  }
  std::vector<M2LLaunch> out;
  if (plans.empty()) return out;
  for (auto& b : B) out.push_back(upload(b, cfg, plans[0]->prec, plans[0]->ip.Kp, ws, s));
  return out;
}

void run_schedule(std::vector<M2LLaunch>& sched, int32_t* heads, int prec, const Interp& ip,
                  const TuneConfig& cfg, hipStream_t s, hipEvent_t* done) {
  if (sched.empty()) return;
  if (cfg.persistent) launch_fill_i32(heads, static_cast<int64_t>(sched.size()), 0, s);
  for (size_t i = 0; i < sched.size(); ++i) {
    const M2LLaunch& L = sched[i];
    if (L.n_gen) launch_bank_matrices(L, prec, ip, s);
    launch_m2l_items(L, prec, ip.Kp, cfg, heads + i, s);
    if (done) FDM_HIP(hipEventRecord(done[i], s));
  }
}

void plan_launch_events(Plan& P) {
  for (hipEvent_t e : P.launch_ev) (void)hipEventDestroy(e);
  P.launch_ev.clear();
  if (!P.timing) return;
  P.launch_ev.resize(P.sched.size(), nullptr);
  for (auto& e : P.launch_ev) FDM_HIP(hipEventCreate(&e));
}

int64_t plan_workspace_bytes(const Plan& P) {
  if (P.bank_budget <= 0 || P.base_items.empty()) return 0;
  const int64_t mb = bank_matrix_bytes(P.prec, P.ip);
  return std::max<int64_t>(1, std::min(P.n_bank, P.bank_budget / mb)) * mb;
}

// Low-rank couplings of one or more plans (one batch): every item's offsets
// ordered by rank (highest first, stable) and cut into groups of 16 (the
// FP32 totals' flush interval); a group runs at the padded rank of its
// first offset.  One launch pair (stage 1, stage 2) covers group g of
// consecutive items, over all plans, while their stage-1 output fits the T
// buffer; T of an item group sits at `compact` units of 64 x 16 complex
// values.  An item with no offset is stored (as zero) by group 0.
std::vector<M2LLaunch> build_aca_schedule(const std::vector<Plan*>& plans,
                                          const TuneConfig& cfg, DevBuf<float>& T,
                                          int64_t T_budget, int64_t* tally, hipStream_t s) {
  constexpr int G = 16;
  if (plans.empty()) return {};
  const int kp = plans[0]->aca_kp, Kp = plans[0]->ip.Kp, prec = plans[0]->prec;
  std::vector<std::vector<int32_t>> vos(plans.size());
  int max_groups = 1;
  for (size_t q = 0; q < plans.size(); ++q) {
    Plan& P = *plans[q];
    std::vector<int32_t>& vo = vos[q];
    vo = P.valid_off_h;  // the low-rank bank stores every matrix at its bank id
    for (const M2LItem& it : P.base_items) {
      std::stable_sort(vo.begin() + it.vo_begin, vo.begin() + it.vo_begin + it.vo_count,
                       [&](int32_t a, int32_t b) { return P.aca_rank[a] > P.aca_rank[b]; });
      max_groups = std::max(max_groups, (it.vo_count + G - 1) / G);
    }
    to_device(P.aca_vo, vo, s, &P.tally);
    P.aca_issued_cols = 0;
  }
  const int64_t cap_units = std::max<int64_t>(G * (kp / 16), T_budget / 8192);
  struct Part {
    int plan;
    M2LItem it;
    int64_t units;
  };
  std::vector<std::vector<Part>> launches;
  int64_t need = 0;
  for (int g = 0; g < max_groups; ++g) {
    std::vector<Part> cur;
    int64_t used = 0;
    for (size_t q = 0; q < plans.size(); ++q) {
      Plan& P = *plans[q];
      for (const M2LItem& base : P.base_items) {
        const int n = std::max(0, std::min(G, base.vo_count - g * G));
        if (n == 0 && g > 0) continue;
        M2LItem it = base;
        it.vo_begin = base.vo_begin + g * G;
        it.vo_count = n;
        int rp = 16;
        if (n) {
          rp = (P.aca_rank[vos[q][it.vo_begin]] + 15) / 16 * 16;
          rp = std::min(std::max(rp, 16), kp);
        }
        it.first = (g == 0 ? 1 : 0) | (rp / 16) << 1;
        const int64_t units = int64_t(n) * (rp / 16);
        P.aca_issued_cols += 64.0 * n * rp;
        if (used + units > cap_units && !cur.empty()) {
          launches.push_back(std::move(cur));
          cur.clear();
          used = 0;
        }
        it.compact = static_cast<int32_t>(used);
        used += units;
        need = std::max(need, used);
        cur.push_back({static_cast<int>(q), it, units});
      }
    }
    if (!cur.empty()) launches.push_back(std::move(cur));
  }
  if (T.size() < static_cast<size_t>(need * 2048)) T.alloc(std::max<int64_t>(need, 1) * 2048, tally);
  std::vector<M2LLaunch> out;
  for (const auto& parts : launches) {
    for (int stage = 1; stage <= 2; ++stage) {
      LaunchBuilder B;
      std::vector<std::vector<int32_t>> desc_of(plans.size());
      for (size_t q = 0; q < plans.size(); ++q) {
        Plan& P = *plans[q];
        desc_of[q].assign(P.levels + 1, -1);
        for (int l = std::max(P.l_min, 0); l <= P.levels; ++l) {
          desc_of[q][l] = static_cast<int32_t>(B.descs.size());
          M2LDesc d = level_desc(P, l, resident_bank(P), 0);
          d.valid_off = P.aca_vo.get();
          if (stage == 1)
            d.out = T.get();  // stage 1 writes T
          else
            d.mom = T.get();  // stage 2 reads it
          B.descs.push_back(d);
        }
      }
      for (const Part& pt : parts) {
        if (stage == 1 && pt.it.vo_count == 0) continue;
        M2LItem it = pt.it;
        it.desc = desc_of[pt.plan][it.desc];
        B.items.push_back(it);
        B.weight.push_back(static_cast<double>(pt.units));
      }
      M2LLaunch L = upload(B, cfg, prec, Kp, nullptr, s);
      L.stage = stage;
      L.resident_wgs = resident_aca(stage, Kp);
      out.push_back(std::move(L));
    }
  }
  return out;
}

void build_plan_schedule(Plan& P, hipStream_t s) {
  if (P.aca_kp) {
    P.sched = build_aca_schedule({&P}, P.tune, P.aca_T, P.aca_T_budget, &P.tally, s);
    P.sched_static.clear();
    P.static_ready = false;
    P.heads.alloc(std::max<size_t>(P.sched.size(), 1), &P.tally);
    P.sched_ready = true;
    plan_launch_events(P);
    return;
  }
  void* ws = nullptr;
  int64_t ws_mats = 0;
  const int64_t ws_bytes = plan_workspace_bytes(P);
  if (ws_bytes > 0) {
    ws_mats = ws_bytes / bank_matrix_bytes(P.prec, P.ip);
    if (P.bank_ws.size() < static_cast<size_t>(ws_bytes)) P.bank_ws.alloc(ws_bytes, &P.tally);
    ws = P.bank_ws.get();
  }
  P.sched = build_schedule({&P}, P.tune, ws, ws_mats, s);
  P.sched_static.clear();
  P.static_ready = false;
  if (ws_bytes > 0 && ws_bytes <= static_workspace_bytes()) {
    // same launches (the schedule depends only on the workspace's matrix
    // count), the bank generated into the static workspace
    P.sched_static = build_schedule({&P}, P.tune, static_workspace(), ws_mats, s);
    P.static_ready = P.sched_static.size() == P.sched.size();
  }
  P.heads.alloc(std::max<size_t>(P.sched.size(), 1), &P.tally);
  P.sched_ready = true;
  plan_launch_events(P);
}

namespace {

// Direction index of -u for the direction u of index c on a level with nd
// directions (Alg. 3 order: 4^k sub-faces per face, faces in -/+ pairs).
int antipodal_direction(int c, int nd) {
  if (nd == 1) return c;
  const int per_face = nd / 6;
  return ((c / per_face) ^ 1) * per_face + c % per_face;
}

// Whether every admissible offset of every coupling level has its partner
// -o at the mirrored position of the sorted list (the admissible set is
// symmetric and sorted lexicographically) with the antipodal direction:
// then A_{-o} = A_o^T (the dir map is odd, readings of the face order).
bool bank_pairs_mirror(const Plan& P) {
  for (int l = std::max(P.l_min, 0); l <= P.levels; ++l) {
    const LevelTable& T = P.tab[l];
    const size_t n = T.adm.size();
    if (n % 2) return false;
    const int nd = direction_count(l, P.l_hf);
    for (size_t i = 0; i < n; ++i) {
      const Off& a = T.adm[i];
      const Off& b = T.adm[n - 1 - i];
      if (b.x != -a.x || b.y != -a.y || b.z != -a.z) return false;
      if (T.dir[n - 1 - i] != antipodal_direction(T.dir[i], nd)) return false;
    }
  }
  return true;
}

}  // namespace

int32_t matrix_code(const Plan& P, int l, size_t i) {
  const int64_t b = P.L[l].bank_base + static_cast<int64_t>(i);
  if (!P.sym) return static_cast<int32_t>(b << 1);
  // stored: the first half of each level's sorted list, in order
  const int64_t n = static_cast<int64_t>(P.tab[l].adm.size());
  const int64_t half_base = P.L[l].bank_base / 2;  // earlier levels hold n / 2 each
  const int64_t j = static_cast<int64_t>(i);
  return j < n / 2 ? static_cast<int32_t>((half_base + j) << 1)
                   : static_cast<int32_t>(((half_base + n - 1 - j) << 1) | 1);
}

void launch_bank(Plan& P, hipStream_t s) {
  // bank id -> (level, offset, direction), for resident and streamed banks
  P.bank_info.clear();
  P.bank_info.reserve(5 * P.n_bank);
  for (int l = 0; l <= P.levels; ++l) {
    if (l < P.l_min) continue;
    const LevelTable& T = P.tab[l];
    for (size_t i = 0; i < T.adm.size(); ++i)
      P.bank_info.insert(P.bank_info.end(), {l, T.adm[i].x, T.adm[i].y, T.adm[i].z, T.dir[i]});
  }
  // (row blocks shift the stored orientation's rows; the transposed reads
  // would need another shift: matrices split into row blocks are all stored)
  P.sym = P.bank_budget == 0 && !P.full_bank && !P.aca_kp && m2l_row_blocks(P.ip.Kp) == 1 &&
          (P.prec == FDM_PREC_FP64 || P.prec == FDM_PREC_FP32) && bank_pairs_mirror(P);
  P.n_bank_stored = 0;
  if (P.n_bank == 0 || P.bank_budget != 0) return;  // streamed: generated per matvec
  std::vector<BankLevel> bl(P.levels + 1);
  for (int l = 0; l <= P.levels; ++l) bl[l] = bank_level(P, l);
  if (P.aca_kp) {  // low-rank bank: the crosses of every stored matrix
    DevBuf<int32_t> d_info, d_rank(P.n_bank);
    DevBuf<BankLevel> d_bl;
    to_device(d_info, P.bank_info, s, nullptr);
    to_device(d_bl, bl, s, nullptr);
    P.aca_bank.alloc(P.n_bank * aca_matrix_bytes(P.ip, P.aca_kp) / 4, &P.tally);
    launch_aca(d_info.get(), P.n_bank, d_bl.get(), P.ip, P.aca_eps, P.aca_kp,
               P.aca_bank.get(), d_rank.get(), s);
    P.aca_rank = to_host(d_rank.get(), P.n_bank, s);
    P.n_bank_stored = P.n_bank;
    return;
  }
  std::vector<int32_t> info;  // the stored matrices, in bank order
  if (P.sym) {
    for (int l = std::max(P.l_min, 0); l <= P.levels; ++l) {
      const size_t n = P.tab[l].adm.size();
      const int64_t b0 = P.L[l].bank_base;
      info.insert(info.end(), P.bank_info.begin() + 5 * b0,
                  P.bank_info.begin() + 5 * (b0 + static_cast<int64_t>(n / 2)));
    }
  } else {
    info = P.bank_info;
  }
  P.n_bank_stored = static_cast<int64_t>(info.size() / 5);
  DevBuf<int32_t> d_info;
  DevBuf<BankLevel> d_bl;
  to_device(d_info, info, s, nullptr);
  to_device(d_bl, bl, s, nullptr);
  const int64_t elems = P.n_bank_stored * bank_matrix_bytes(P.prec, P.ip);
  void* dst = nullptr;
  if (P.prec == FDM_PREC_FP64) {
    P.bank64.alloc(elems / 8, &P.tally);
    dst = P.bank64.get();
  } else if (P.prec == FDM_PREC_BF16X3 || P.prec == FDM_PREC_BF16X6) {
    P.bank16.alloc(elems / 2, &P.tally);
    dst = P.bank16.get();
  } else {
    P.bank32.alloc(elems / 4, &P.tally);
    dst = P.bank32.get();
  }
  launch_bank_direct(d_info.get(), P.n_bank_stored, d_bl.get(), P.prec, P.ip, dst, s);
  FDM_HIP(hipStreamSynchronize(s));
}

void build_m2l_work(Plan& P, hipStream_t s) {
  const int p = P.levels;
  const int nb = P.tune.nb;
  std::vector<M2LItem> items;
  std::vector<int32_t> tgt_list, cand, cand_begin_per_item, cand_count_per_item;
  std::vector<int4> offtab(P.n_bank);
  for (int l = 0; l <= p; ++l) {
    const LevelTable& T = P.tab[l];
    LevelData& Ld = P.L[l];
    if (l < P.l_min) continue;
    for (size_t i = 0; i < T.adm.size(); ++i)
      offtab[Ld.bank_base + i] = make_int4(T.adm[i].x, T.adm[i].y, T.adm[i].z,
                                           matrix_code(P, l, i));
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
    for (size_t b = 0; b < keys.size(); ++b)  // (adaptive trees: boxes that exist)
      if (!P.adaptive() || P.stateT_h[l][b] != 0)
        by_oct[keys[b] & 7].push_back(static_cast<int32_t>(b));
    // items ordered (octant, direction, block): one group per (octant,
    // direction), blocks in Morton order within a group
    for (int q = 0; q < 8; ++q) {
      const auto& bx = by_oct[q];
      std::vector<std::pair<int32_t, int32_t>> blocks;  // (tgt_begin, ntgt)
      for (size_t b0 = 0; b0 < bx.size(); b0 += nb) {
        const int nt = static_cast<int>(std::min<size_t>(nb, bx.size() - b0));
        blocks.push_back({static_cast<int32_t>(tgt_list.size()), nt});
        tgt_list.insert(tgt_list.end(), bx.begin() + b0, bx.begin() + b0 + nt);
      }
      for (int c = 0; c < Ld.nd; ++c)
        for (auto [tb, nt] : blocks) {
          items.push_back(M2LItem{l, c, tb, nt, 0, 0, 1, 0});
          cand_begin_per_item.push_back(list_begin[q * Ld.nd + c]);
          cand_count_per_item.push_back(static_cast<int32_t>(lists[q * Ld.nd + c].size()));
        }
    }
  }
  const int64_t n_items = static_cast<int64_t>(items.size());
  P.offtab.alloc(std::max<int64_t>(P.n_bank, 1), &P.tally);
  if (P.n_bank)
    FDM_HIP(hipMemcpyAsync(P.offtab.get(), offtab.data(), offtab.size() * sizeof(int4),
                           hipMemcpyHostToDevice, s));
  to_device(P.tgt_list, tgt_list, s, &P.tally);
  P.base_items.clear();
  P.valid_off_h.clear();
  P.sched.clear();
  P.sched_static.clear();
  P.static_ready = false;
  P.sched_ready = false;
  P.item_tiles.clear();
  if (n_items == 0) {
    P.valid_off.alloc(1, &P.tally);
    FDM_HIP(hipStreamSynchronize(s));
    return;
  }
  std::vector<M2LDesc> descs(p + 1);
  for (int l = 0; l <= p; ++l) descs[l] = level_desc(P, l, nullptr, 0);
  DevBuf<M2LDesc> d_descs;
  to_device(d_descs, descs, s, nullptr);
  DevBuf<M2LItem> d_items;
  DevBuf<int32_t> d_cand, d_cb, d_cc, d_counts(n_items), d_begin;
  to_device(d_items, items, s, nullptr);
  to_device(d_cand, cand, s, nullptr);
  to_device(d_cb, cand_begin_per_item, s, nullptr);
  to_device(d_cc, cand_count_per_item, s, nullptr);
  DevBuf<unsigned long long> d_bpo(std::max<int64_t>(P.n_bank, 1));
  DevBuf<int32_t> d_tiles(n_items);
  FDM_HIP(hipMemsetAsync(d_bpo.get(), 0, d_bpo.bytes(), s));
  launch_valid_offsets(d_items.get(), n_items, d_cb.get(), d_cc.get(), d_cand.get(),
                       d_descs.get(), P.tgt_list.get(), P.offtab.get(), 0, d_counts.get(),
                       nullptr, nullptr, nullptr, nullptr, s);
  std::vector<int32_t> counts = to_host(d_counts.get(), n_items, s);
  std::vector<int32_t> begin(n_items);
  int64_t total = 0;
  for (int64_t i = 0; i < n_items; ++i) {
    begin[i] = static_cast<int32_t>(total);
    total += counts[i];
  }
  if (total > INT32_MAX) fail(FDM_ERR_UNSUPPORTED, "coupling work list too long");
  to_device(d_begin, begin, s, nullptr);
  P.valid_off.alloc(std::max<int64_t>(total, 1), &P.tally);
  launch_valid_offsets(d_items.get(), n_items, d_cb.get(), d_cc.get(), d_cand.get(),
                       d_descs.get(), P.tgt_list.get(), P.offtab.get(), 1, nullptr,
                       d_begin.get(), P.valid_off.get(), d_bpo.get(), d_tiles.get(), s);
  std::vector<unsigned long long> bpo = to_host(d_bpo.get(), P.n_bank, s);
  P.item_tiles = to_host(d_tiles.get(), n_items, s);
  P.bank_work.assign(bpo.begin(), bpo.end());
  P.valid_off_h = to_host(P.valid_off.get(), total, s);
  for (int64_t i = 0; i < n_items; ++i) {
    items[i].vo_begin = begin[i];
    items[i].vo_count = counts[i];
  }
  P.base_items = std::move(items);
  // statistics and per-level offset use for export
  P.n_couplings = 0;
  P.n_stored = 0;
  P.off_used.assign(p + 1, {});
  for (int l = 0; l <= p; ++l) {
    if (l < P.l_min) continue;
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

}  // namespace fdm
