// The plan: trees, block-partition tables, direction tables, coupling bank
// and the workspaces of one fast directional matvec.
#pragma once

#include <array>
#include <string>

#include "kernels.hpp"

namespace fdm {

struct Off {
  int x, y, z;
  bool operator<(const Off& o) const {
    if (x != o.x) return x < o.x;
    if (y != o.y) return y < o.y;
    return z < o.z;
  }
  bool operator==(const Off& o) const { return x == o.x && y == o.y && z == o.z; }
};

// Host tables of one level (Sect. 2.3/2.4), independent of the points:
// offsets o = i_t - i_s of same-level box pairs whose parent pair was
// refined, split into admissible ones (with the set of target octants for
// which the parent pair was refined) and inadmissible ones.
struct LevelTable {
  std::vector<Off> adm;
  std::vector<uint8_t> mask;    // bit q: target octant q reaches this offset
  std::vector<int32_t> dir;     // direction index c_(l)(t,s)
  std::vector<Off> inadm;
};

std::vector<LevelTable> build_level_tables(double kappa, double side, int levels,
                                           int l_hf, double eta2);
int direction_index(int level, int l_hf, const Off& o);
std::vector<double> direction_vectors(int level, int l_hf);  // nd * 3
int direction_count(int level, int l_hf);

// Coupling-kernel work item: one block of <= kNB target boxes of one octant
// on one level, for one direction, with its list of offsets that hit at
// least one non-empty source box.
constexpr int kNB = 64;
// One wave per 32 padded rows: Kp <= 384, i.e. m <= 6, in the coupling kernels.
constexpr int kM2LMaxThreads = 768;
constexpr int kMaxKp = kM2LMaxThreads / 2;
struct M2LItem {
  int32_t level;
  int32_t c;
  int32_t tgt_begin;  // into tgt_list
  int32_t ntgt;
  int32_t vo_begin;   // into valid_off
  int32_t vo_count;
};

// Per-level device view used by the coupling kernel.
struct M2LLevel {
  const int32_t* gridS;   // source box grid of the level
  const uint32_t* keyT;   // target box keys
  const void* mom;        // operand moments [nbS][nd][Kp] complex
  void* out;              // coupling result [nbT][nd][Kp] complex
  int32_t nd;
  int32_t level;
};

struct LevelData {
  int level = 0;
  int nd = 1;          // #D^(l) (1 on low-frequency levels)
  double h = 0;        // box side
  int64_t bank_base = 0;  // bank id of adm[0]
  DevBuf<double> dirvec;  // nd * 3
  DevBuf<int32_t> offs;   // adm offsets: x, y, z, bank id
  // moments / locals, complex, [nb][nd][Kp]
  DevBuf<double> mom64;   // FP64 moments (all precisions)
  DevBuf<float> mom32;    // FP32 operand copy (mixed precisions)
  DevBuf<double> loc64;   // FP64 locals (coupling result + parent transfer)
};

struct Plan {
  int64_t nT = 0, nS = 0;
  double kappa = 0;
  double lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
  double side = 0;
  int levels = 0, m = 0, prec = 0;
  int l_hf = -1, l_min = 0;
  double eta2 = 5.0;
  Interp ip;
  int64_t tally = 0;  // device bytes held

  DevTree T, S;
  std::vector<LevelTable> tab;
  std::vector<LevelData> L;  // index = level

  // coupling bank: one K x K complex matrix per admissible (level, offset)
  int64_t n_bank = 0;
  DevBuf<double> bank64;
  DevBuf<float> bank32;
  DevBuf<uint16_t> bank16;

  // coupling work
  DevBuf<M2LItem> items;
  DevBuf<int32_t> tgt_list, valid_off;
  DevBuf<M2LLevel> m2l_levels;
  DevBuf<int4> offtab;  // per bank matrix: offset x, y, z and bank id
  int64_t n_items = 0;

  // near field
  DevBuf<int32_t> near_off;  // x, y, z triples at the leaf level
  int n_near_off = 0;

  // workspaces
  DevBuf<double> v_tree;  // complex128 [nS]
  DevBuf<double> y_tree;  // complex128 [nT]
  DevBuf<double> io64;    // complex128 staging for complex64 I/O

  // statistics
  int64_t n_couplings = 0, n_stored = 0, near_pairs = 0, near_entries = 0;
  int64_t m2l_columns = 0;
  double setup_ms = 0;
  bool has_run = false;

  // optional per-phase timing (events on the matvec stream)
  bool timing = false, timed_run = false;
  hipEvent_t ev[8] = {};

  // structure export (host copies made at build time)
  std::vector<std::vector<int64_t>> off_used;  // per level: x,y,z,count,dir
};

void plan_build(Plan& P, const double* pT, const double* pS, hipStream_t s);
// v_user / y_user are complex128, or complex64 when c64 is set.
void plan_matvec(Plan& P, const void* v_user, void* y_user, bool c64, hipStream_t s);

// kernel launchers (upward.hip, downward.hip, nearfield.hip, m2l.hip)
void launch_permute_in(const double* v_user, const int32_t* perm, int64_t n,
                       double* v_tree, hipStream_t s);
void launch_permute_out(const double* y_tree, const int32_t* perm, int64_t n,
                        double* y_user, hipStream_t s);
void launch_permute_in_c64(const float* v_user, const int32_t* perm, int64_t n,
                           double* v_tree, hipStream_t s);
void launch_permute_out_c64(const double* y_tree, const int32_t* perm, int64_t n,
                            float* y_user, hipStream_t s);
void launch_s2m(Plan& P, hipStream_t s);
void launch_m2m(Plan& P, int level, hipStream_t s);
void launch_l2l(Plan& P, int level, hipStream_t s);
void launch_zero_c128(double* p, int64_t n, hipStream_t s);
void launch_l2t(Plan& P, hipStream_t s);
void launch_p2p(Plan& P, hipStream_t s);
void launch_bank(Plan& P, hipStream_t s);
void launch_m2l(Plan& P, hipStream_t s);
void build_m2l_work(Plan& P, hipStream_t s);
void launch_dense(const double* pT, int64_t nT, const double* pS, int64_t nS,
                  double kappa, const double* v, double* y, hipStream_t s);

}  // namespace fdm

// The opaque handle of the C ABI.
struct fdm_plan {
  fdm::Plan p;
};
