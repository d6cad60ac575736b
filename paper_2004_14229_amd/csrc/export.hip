// Named host copies of plan arrays (fdm_plan_export): tree structure, the
// block partition's offsets and direction sets, and the moments / locals of
// the last matvec, for parity checks against an independent implementation.
#include <cctype>
#include <cstdlib>
#include <cstring>
#include <set>
#include <string>

#include "plan.hpp"

namespace fdm {

namespace {

std::vector<int64_t> widen_i32(const int32_t* d, size_t n) {
  std::vector<int32_t> h = to_host(d, n, nullptr);
  return std::vector<int64_t>(h.begin(), h.end());
}

std::vector<int64_t> widen_u32(const uint32_t* d, size_t n) {
  std::vector<uint32_t> h = to_host(d, n, nullptr);
  return std::vector<int64_t>(h.begin(), h.end());
}

// Active directions D(t) (target side) or D(s) (source side) per box of a
// level: the direction indices of the admissible blocks the box takes part in.
std::vector<std::set<int>> active_dirs(const Plan& P, int l, bool target) {
  const DevTree& A = target ? P.T : P.S;  // boxes whose sets are formed
  const DevTree& B = target ? P.S : P.T;  // partner boxes
  std::vector<std::set<int>> D(A.nb[l]);
  if (A.nb[l] == 0 || B.nb[l] == 0 || l < P.l_min) return D;
  std::vector<uint32_t> keys = to_host(A.key[l].get(), A.nb[l], nullptr);
  std::vector<int32_t> grid = to_host(B.grid[l].get(), size_t(1) << (3 * l), nullptr);
  if (P.adaptive()) {  // only boxes that exist in the adaptive trees
    const auto& sb = target ? P.stateS_h[l] : P.stateT_h[l];
    for (auto& g : grid)
      if (g >= 0 && sb[g] == 0) g = -1;
  }
  const auto* sa = P.adaptive() ? &(target ? P.stateT_h : P.stateS_h)[l] : nullptr;
  const LevelTable& T = P.tab[l];
  const int lim = 1 << l;
  for (size_t b = 0; b < keys.size(); ++b) {
    if (sa && (*sa)[b] == 0) continue;
    int ix, iy, iz;
    demorton3(keys[b], l, ix, iy, iz);
    for (size_t i = 0; i < T.adm.size(); ++i) {
      const int sg = target ? -1 : 1;  // partner = box -/+ o
      const int px = ix + sg * T.adm[i].x, py = iy + sg * T.adm[i].y, pz = iz + sg * T.adm[i].z;
      if (px < 0 || py < 0 || pz < 0 || px >= lim || py >= lim || pz >= lim) continue;
      if (grid[morton3(px, py, pz, l)] < 0) continue;
      const int q = target ? int(keys[b] & 7) : ((px & 1) << 2) | ((py & 1) << 1) | (pz & 1);
      if (!(T.mask[i] & (1u << q))) continue;
      D[b].insert(T.dir[i]);
    }
  }
  return D;
}

// Codes box * nd + c; with `state` (adaptive trees) boxes are numbered
// among those that exist.
std::vector<int64_t> dir_codes(const std::vector<std::set<int>>& D, int nd,
                               const std::vector<uint8_t>* state = nullptr) {
  std::vector<int64_t> out;
  int64_t idx = 0;
  for (size_t b = 0; b < D.size(); ++b) {
    if (state && (*state)[b] == 0) continue;
    for (int c : D[b]) out.push_back(idx * nd + c);
    ++idx;
  }
  return out;
}

// Values of the boxes that exist in the adaptive trees (all for uniform ones).
std::vector<int64_t> existing(const Plan& P, const std::vector<int64_t>& v, bool target, int l) {
  if (!P.adaptive()) return v;
  const auto& st = (target ? P.stateT_h : P.stateS_h)[l];
  std::vector<int64_t> out;
  for (size_t b = 0; b < v.size(); ++b)
    if (st[b] != 0) out.push_back(v[b]);
  return out;
}

std::vector<int64_t> export_int(const Plan& P, const std::string& name, bool& found) {
  found = true;
  auto lev = [&](size_t prefix) { return std::atoi(name.c_str() + prefix); };
  if (name == "perm_T") return widen_i32(P.T.perm.get(), P.nT);
  if (name == "perm_S") return widen_i32(P.S.perm.get(), P.nS);
  if (name == "l_hf") return {P.l_hf};
  if (name == "near_pairs") return {P.near_pairs};
  if (name == "aca_rank") return std::vector<int64_t>(P.aca_rank.begin(), P.aca_rank.end());
  if (name == "bank_offsets")
    return std::vector<int64_t>(P.bank_info.begin(), P.bank_info.end());
  if (name == "near_entries") return {P.near_entries};
  for (const char* tag : {"T", "S"}) {
    const DevTree& A = tag[0] == 'T' ? P.T : P.S;
    for (const char* what : {"keys_", "start_", "count_"}) {
      std::string pre = std::string(what) + tag;
      if (name.compare(0, pre.size(), pre) == 0 && name.size() > pre.size()) {
        int l = lev(pre.size());
        if (l < 0 || l > P.levels) break;
        if (A.n == 0) return {};
        const bool tg = tag[0] == 'T';
        if (what[0] == 'k') return existing(P, widen_u32(A.key[l].get(), A.nb[l]), tg, l);
        if (what[0] == 's') return existing(P, widen_i32(A.start[l].get(), A.nb[l]), tg, l);
        return existing(P, widen_i32(A.count[l].get(), A.nb[l]), tg, l);
      }
    }
  }
  for (const char* what : {"nc_", "off_", "offdir_", "offcnt_"}) {
    std::string pre(what);
    if (name.compare(0, pre.size(), pre) == 0) {
      int l = lev(pre.size());
      if (l < 0 || l > P.levels) break;
      std::vector<int64_t> out;
      int64_t nc = 0;
      if (l < static_cast<int>(P.off_used.size())) {
        const auto& u = P.off_used[l];
        for (size_t i = 0; i + 5 <= u.size(); i += 5) {
          if (pre == "off_") {
            out.push_back(u[i]);
            out.push_back(u[i + 1]);
            out.push_back(u[i + 2]);
          } else if (pre == "offcnt_") {
            out.push_back(u[i + 3]);
          } else if (pre == "offdir_") {
            out.push_back(u[i + 4]);
          }
          nc += u[i + 3];
        }
      }
      if (pre == "nc_") return {nc};
      return out;
    }
  }
  for (const char* tag : {"D_T", "D_S", "Dh_T", "Dh_S"}) {
    std::string pre(tag);
    if (name.compare(0, pre.size(), pre) == 0 && name.size() > pre.size() &&
        std::isdigit(static_cast<unsigned char>(name[pre.size()]))) {
      int l = lev(pre.size());
      if (l < 0 || l > P.levels) break;
      const bool target = pre.back() == 'T';
      const int nd = direction_count(l, P.l_hf);
      const std::vector<uint8_t>* st =
          P.adaptive() ? &(target ? P.stateT_h : P.stateS_h)[l] : nullptr;
      if (pre[1] != 'h') return dir_codes(active_dirs(P, l, target), nd, st);
      // inherited: D^(t) = { dir_(l)(c) : c in D(t') u D^(t'), t' = parent(t) }
      const DevTree& A = target ? P.T : P.S;
      std::vector<std::set<int>> up;  // D u D^ of the boxes one level up
      for (int k = 0; k <= l; ++k) {
        std::vector<std::set<int>> Dk = active_dirs(P, k, target);
        std::vector<std::set<int>> Dh(A.nb[k]);
        if (k > 0 && A.nb[k]) {
          std::vector<uint32_t> keys = to_host(A.key[k].get(), A.nb[k], nullptr);
          std::vector<int32_t> pgrid = to_host(A.grid[k - 1].get(), size_t(1) << (3 * (k - 1)), nullptr);
          for (size_t b = 0; b < keys.size(); ++b) {
            int par = pgrid[keys[b] >> 3];
            for (int c : up[par]) Dh[b].insert(k <= P.l_hf ? (c >> 2) : 0);
          }
        }
        if (k == l) return dir_codes(Dh, nd, st);
        up.assign(A.nb[k], {});
        for (size_t b = 0; b < Dk.size(); ++b) {
          up[b] = Dk[b];
          up[b].insert(Dh[b].begin(), Dh[b].end());
        }
      }
    }
  }
  found = false;
  return {};
}

// Complex coefficients of one level (moments or locals), padding stripped.
std::vector<double> export_coeffs(const Plan& P, int l, bool locals) {
  if (l < P.l_min || l > P.levels) return {};
  const LevelData& Ld = P.L[l];
  const DevTree& A = locals ? P.T : P.S;
  const int64_t nv = A.nb[l] * int64_t(Ld.nd);
  const int K = P.ip.K, Kp = P.ip.Kp;
  std::vector<double> raw = to_host(locals ? Ld.loc64.get() : Ld.mom64.get(), 2 * nv * Kp, nullptr);
  std::vector<double> out(2 * nv * K);
  for (int64_t v = 0; v < nv; ++v)
    for (int k = 0; k < K; ++k) {
      out[2 * (v * K + k)] = raw[2 * (v * Kp + k)];
      out[2 * (v * K + k) + 1] = raw[2 * (v * Kp + k) + 1];
    }
  return out;
}

}  // namespace

}  // namespace fdm

using namespace fdm;

extern "C" int fdm_plan_export(const fdm_plan* plan, const char* name, void* host,
                               int64_t capacity, int64_t* size) {
  try {
    if (!plan || !name || !size) return FDM_ERR_INVALID_ARG;
    const Plan& P = plan->p;
    const std::string n(name);
    std::vector<int64_t> iv;
    std::vector<double> dv;
    bool is_double = false, found = true;
    auto level_of = [&](size_t pre) { return std::atoi(n.c_str() + pre); };
    if (n.compare(0, 5, "dirs_") == 0) {
      int l = level_of(5);
      if (l < 0 || l > P.levels) return FDM_ERR_INVALID_ARG;
      dv = direction_vectors(l, P.l_hf);
      is_double = true;
    } else if (n.compare(0, 4, "mom_") == 0 || n.compare(0, 4, "loc_") == 0) {
      if (!P.has_run) return FDM_ERR_STATE;
      FDM_HIP(hipDeviceSynchronize());
      dv = export_coeffs(P, level_of(4), n[0] == 'l');
      is_double = true;
    } else {
      iv = export_int(P, n, found);
    }
    if (!found) return FDM_ERR_INVALID_ARG;
    const int64_t bytes = is_double ? int64_t(dv.size() * sizeof(double))
                                    : int64_t(iv.size() * sizeof(int64_t));
    *size = bytes;
    if (!host) return FDM_OK;
    if (capacity < bytes) return FDM_ERR_INVALID_ARG;
    if (bytes) std::memcpy(host, is_double ? static_cast<const void*>(dv.data())
                                           : static_cast<const void*>(iv.data()), bytes);
    return FDM_OK;
  } catch (const Error& e) {
    return e.status;
  } catch (...) {
    return FDM_ERR_STATE;
  }
}
