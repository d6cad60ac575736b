// The plan: trees, block-partition tables, direction tables, coupling bank
// and the workspaces of one fast directional matvec; and the batch of plans
// whose coupling and near-field work runs from one device queue.
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

// side: the root box's three side lengths.
std::vector<LevelTable> build_level_tables(double kappa, const double side[3], int levels,
                                           int l_hf, double eta2);
// dir_(level) of the centre offset o * h of two boxes of one level; scale:
// the box sides as integers up to one common factor ({1, 1, 1} for cubes).
int direction_index(int level, int l_hf, const Off& o, const int64_t scale[3]);
int direction_index(int level, int l_hf, const Off& o);  // cubic boxes
// The root box's sides as integers up to one common positive factor (exact:
// the doubles' odd mantissas shifted to a common exponent); throws
// FDM_ERR_UNSUPPORTED when that does not fit 63 bits.
void side_scale(const double side[3], int64_t scale[3]);
std::vector<double> direction_vectors(int level, int l_hf);  // nd * 3
int direction_count(int level, int l_hf);

// ------------------------------------------------------- coupling work --
// A coupling work item is a block of <= nb target boxes (nb = 32 or 64) of
// one octant on one level, for one direction, with the list of offsets that
// hit at least one non-empty source box.  One wave per 32 padded rows, at
// most 384 rows (12 waves) per workgroup: a matrix with more rows (m = 7,
// 8: Kp = 512, 736) runs each item once per row block.
constexpr int kMaxNB = 64;
constexpr int kM2LMaxThreads = 768;
constexpr int kMaxKp = kM2LMaxThreads / 2;  // rows per workgroup

// Descriptor of one (plan, level) of a coupling launch.
struct M2LDesc {
  const int32_t* gridS;      // source box grid of the level
  const uint32_t* keyT;      // target box keys of the level
  const void* mom;           // operand moments [nbS][nd][Kp] complex
  void* out;                 // FP64 result [nbT][nd][Kp] complex
  const int32_t* tgt_list;   // target boxes of the plan's items
  const int32_t* valid_off;  // bank ids of the plan's items' offsets
  const int4* offtab;        // per bank id: offset x, y, z, (matrix << 1) | transposed
  // bank id b is matrix b counted from `bank`; for a workspace holding a
  // range of ids this address lies before the workspace (never read there)
  const void* bank;
  int32_t nd, level;
  int32_t K;  // interpolation nodes per box, (m+1)^3 <= Kp: rows / k beyond are padding
  int32_t kp;  // low-rank couplings: the rank cap (columns of U, rows of Vt), else 0
  // coupling-matrix rows this descriptor's items compute (Kp; for a matrix
  // split into row blocks, the block's rows: bank and out then point at the
  // block's first row, the row stride stays Kp)
  int32_t rows;
};

// Descriptor of one plan's near field in a queued launch.
struct P2PDesc {
  const double *xt, *yt, *zt;
  const int32_t* leaf_of;
  const uint32_t* keyT;  // leaf keys of the target tree
  const double *xs, *ys, *zs;
  const double* v;       // complex128 charges, tree order
  const int32_t *startS, *countS, *gridS;
  const int32_t* near_off;
  double* y;             // complex128 result, tree order (stored)
  double kappa;
  int32_t n_off, level;
};

// Queue item.  desc >= 0: coupling item of descriptor `desc` -- targets
// tgt_list[tgt_begin .. +ntgt), direction c, offsets valid_off[vo_begin ..
// +vo_count); bit 0 of `first` = 1 for the first part of a (target block,
// c), whose result is stored, 0 for later parts (streamed banks, offset
// groups), which add to it.  `compact` = 1: the coupling item runs with
// compacted columns (FP32 and BF16 kernels, 64 targets per item).
// Low-rank stage items (offset groups of at most 16): `first` >> 1 = the
// group's padded rank / 16, `compact` = its place in the first stage's
// output (units of 64 x 16 complex values).  desc < 0: near-field item of
// P2P descriptor -desc-1 for target points tgt_begin .. +ntgt (tree order).
struct M2LItem {
  int32_t desc, c, tgt_begin, ntgt, vo_begin, vo_count, first, compact;
};

// One matrix to generate into a streamed bank: level descriptor index,
// offset and direction.
struct BankLevel {
  const double* dirvec;
  double h[3];  // box sides of the level
  double kappa;
  int32_t level, nd;
};

// Launch shape and order picked by the autotuner.
struct TuneConfig {
  int nb = 64;           // target boxes per coupling item (32 or 64)
  int persistent = 1;    // 1: persistent workgroups pulling from a device queue
  int lpt = 1;           // 1: heaviest items first; 0: (level, octant, direction, block)
  int p2p_in_queue = 0;  // near-field items in the coupling launch
  int compact = 1;       // column compaction: 0 never, 1 sparse items, 2 every item
};

// One coupling launch: optional bank generation into a workspace, then the
// queue of items over the descriptors.
struct M2LLaunch {
  int64_t n_gen = 0;
  DevBuf<int32_t> gen_info;     // per matrix: bank level index, ox, oy, oz, c
  DevBuf<BankLevel> gen_levels;
  void* gen_dst = nullptr;      // workspace (matrices in gen order)
  int64_t n_items = 0, n_p2p_items = 0;
  int64_t resident_wgs = 0;     // grid of the persistent launch
  bool has_parts = false;       // holds later parts of split items
  int stage = 0;                // low-rank couplings: 1 T = Vt M, 2 g += U T; 0 dense
  DevBuf<M2LItem> items;
  DevBuf<M2LDesc> descs;
  DevBuf<P2PDesc> p2p;
};

struct LevelData {
  int level = 0;
  int nd = 1;          // #D^(l) (1 on low-frequency levels)
  double h[3] = {0, 0, 0};  // box sides
  double3 hv() const { return make_double3(h[0], h[1], h[2]); }
  int64_t bank_base = 0;  // bank id of adm[0]
  DevBuf<double> dirvec;  // nd * 3
  DevBuf<int32_t> offs;   // adm offsets: x, y, z, bank id
  // moments / locals, complex, [nb][nd][Kp]
  DevBuf<double> mom64;   // FP64 moments (all precisions)
  DevBuf<float> mom32;    // FP32 operand copy (FP32, BF16X3)
  // BF16X6 operand copy: per (box, direction) column and slab of 16 k, the
  // six BF16 part planes (re hi, mid, lo, im hi, mid, lo) of 16 values
  DevBuf<uint16_t> mom16;
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

  // coupling bank: one K x K complex matrix per admissible (level, offset),
  // resident, or generated chunk by chunk into a workspace of at most
  // bank_budget bytes during each matvec (streamed)
  int64_t n_bank = 0;
  int64_t bank_budget = 0;  // 0: resident
  // resident FP64 / FP32 bank stored once per offset pair (o, -o): the
  // matrix of -o is applied as the transpose of that of o (Sect. 2.7)
  bool full_bank = false;   // option: store every matrix
  bool sym = false;
  int64_t n_bank_stored = 0;  // matrices in the resident bank
  // low-rank couplings (ACA, Sect. 2.7): per bank id the crosses of its
  // matrix as U (Kp x kp) and Vt (kp x Kp), FP32, and the rank reached; the
  // coupling step runs two stages per launch pair of offset groups, T of a
  // launch pair in aca_T
  double aca_eps = 0;       // 0: dense couplings
  int aca_kp = 0;           // rank cap (32 or 64)
  DevBuf<float> aca_bank;
  std::vector<int32_t> aca_rank;
  DevBuf<float> aca_T;
  DevBuf<int32_t> aca_vo;  // the items' offsets, each item's by rank (highest first)
  double aca_issued_cols = 0;  // sum over groups of offsets x 64 slots x padded rank
  int64_t aca_T_budget = int64_t(8) << 30;  // bytes of T per launch pair
  DevBuf<double> bank64;
  DevBuf<float> bank32;
  DevBuf<uint16_t> bank16;
  DevBuf<uint8_t> bank_ws;
  std::vector<int32_t> bank_info;  // per bank id: level, ox, oy, oz, c
  std::vector<int64_t> bank_work;  // per bank id: admissible blocks using it
  // per base item: the 32-column tiles its offsets take when compacted
  std::vector<int32_t> item_tiles;

  // coupling work (per plan; a batch builds its own launches from it)
  TuneConfig tune;
  std::vector<M2LItem> base_items;  // desc = level, first = 1, in build order
  std::vector<int32_t> valid_off_h;
  DevBuf<int32_t> tgt_list, valid_off;
  // per bank id: offset x, y, z and the matrix applied, (index << 1) | t:
  // stored matrix `index` counted from the bank base, t = 1 transposed
  DevBuf<int4> offtab;
  std::vector<M2LLaunch> sched;
  DevBuf<int32_t> heads;  // one queue head per launch
  bool sched_ready = false;
  // the same launches with the streamed bank generated into the library's
  // static workspace instead of bank_ws (built with sched when the plan's
  // workspace fits it; used by the allocation-free matvec)
  std::vector<M2LLaunch> sched_static;
  bool static_ready = false;
  const void* batch_owner = nullptr;  // the batch holding this plan, if any

  // near field
  DevBuf<int32_t> near_off;  // x, y, z triples at the leaf level
  int n_near_off = 0;

  // adaptive trees (Alg. 1's stop rule, n_max > 0).  The device trees stay
  // refined to the full depth; a box exists in the adaptive tree when every
  // ancestor holds more than n_max points.  Per level and box: 0 pruned,
  // 1 refined, 2 leaf.  Work on pruned boxes is either never issued
  // (couplings, near field, L2T) or computed and never read (moments and
  // locals of the full-depth pass).
  int64_t n_max = 0;
  std::vector<std::vector<uint8_t>> stateT_h, stateS_h;
  std::vector<DevBuf<uint8_t>> stateT, stateS;
  std::vector<DevBuf<int32_t>> gridS_alive;  // source grid without pruned boxes
  std::vector<DevBuf<int32_t>> leafT, leafS;  // per level: leaf boxes
  std::vector<int64_t> n_leafT, n_leafS;
  // near field: one item per (level, existing target box, chunk of at most
  // 256 of its points), x = first point (tree order), y = count | level << 16,
  // [z, w) = its near-field blocks in near_ranges as (first source slot,
  // count); per point the level of its leaf; per level and point the sum of
  // that level's blocks (near_z, complex128 [(levels + 1) * nT])
  DevBuf<int4> near_items;
  DevBuf<int2> near_ranges;
  DevBuf<uint8_t> near_leaf_level;
  DevBuf<double> near_z;
  int64_t n_near_items = 0;
  bool adaptive() const { return n_max > 0; }

  // workspaces
  DevBuf<double> v_tree;  // complex128 [nS]
  DevBuf<double> y_tree;  // complex128 [nT]
  // several right-hand sides (fdm_plan_matvec_multi): all of them in tree
  // order, and the vector the phases of one pass read and write
  DevBuf<double> vm_tree, ym_tree;  // complex128 [nrhs][nS], [nrhs][nT]
  double* v_view = nullptr;
  double* y_view = nullptr;
  double* vtree() const { return v_view ? v_view : v_tree.get(); }
  double* ytree() const { return y_view ? y_view : y_tree.get(); }

  // statistics
  int64_t n_couplings = 0, n_stored = 0, near_pairs = 0, near_entries = 0;
  double setup_ms = 0;
  bool has_run = false;

  // optional per-phase timing (events on the matvec stream)
  bool timing = false, timed_run = false;
  hipEvent_t ev[8] = {};
  std::vector<hipEvent_t> launch_ev;  // one per coupling launch (timing on)

  // structure export (host copies made at build time)
  std::vector<std::vector<int64_t>> off_used;  // per level: x,y,z,count,dir
};

void plan_build(Plan& P, const double* pT, const double* pS, hipStream_t s);
// v_user / y_user are complex128, or complex64 when c64 is set.
// use_static: run the launches of sched_static (the plan must be prepared).
void plan_matvec(Plan& P, const void* v_user, void* y_user, bool c64, hipStream_t s,
                 bool use_static = false);
// The parts of a matvec around the coupling launches (batched matvecs).
void plan_upward(Plan& P, const void* v_user, bool c64, hipStream_t s);
void plan_downward(Plan& P, void* y_user, bool c64, hipStream_t s);
void plan_zero_output(Plan& P, void* y_user, bool c64, hipStream_t s);
void plan_m2m_level(Plan& P, int l, hipStream_t s);
bool p2p_queued(const Plan& P, const TuneConfig& t);

// ------------------------------------------------------------ kernels --
void launch_permute_in(const double* v_user, const int32_t* perm, int64_t n,
                       double* v_tree, hipStream_t s);
void launch_permute_out(const double* y_tree, const int32_t* perm, int64_t n,
                        double* y_user, hipStream_t s);
void launch_permute_in_c64(const float* v_user, const int32_t* perm, int64_t n,
                           double* v_tree, hipStream_t s);
void launch_permute_out_c64(const double* y_tree, const int32_t* perm, int64_t n,
                            float* y_user, hipStream_t s);
void launch_s2m(Plan& P, hipStream_t s);
// S2M / L2T of the listed boxes of one level (adaptive trees: its leaves)
void launch_s2m_boxes(Plan& P, int level, const int32_t* boxes, int64_t n, hipStream_t s);
void launch_l2t_boxes(Plan& P, int level, const int32_t* boxes, int64_t n, hipStream_t s);
void launch_m2m(Plan& P, int level, hipStream_t s);
void launch_l2l(Plan& P, int level, hipStream_t s);
void launch_zero_c128(double* p, int64_t n, hipStream_t s);
void launch_fill_i32(int32_t* p, int64_t n, int32_t value, hipStream_t s);
void launch_l2t(Plan& P, hipStream_t s);  // adds the far field to y_tree
void launch_p2p(Plan& P, hipStream_t s);  // stores the near field into y_tree
void launch_dense(const double* pT, int64_t nT, const double* pS, int64_t nS,
                  double kappa, const double* v, double* y, hipStream_t s);
P2PDesc p2p_desc(const Plan& P);
// adaptive trees (adaptive.hip): box states, leaf lists and pruned grids
// after the full-depth trees are built; near-field statistics; near field
void build_adaptive(Plan& P, hipStream_t s);
void adaptive_near_field(Plan& P, hipStream_t s);  // near-field lists and statistics
void launch_p2p_adaptive(Plan& P, hipStream_t s);

// coupling work and schedules (m2l_work.hip)
void launch_bank(Plan& P, hipStream_t s);  // resident bank
void build_m2l_work(Plan& P, hipStream_t s);  // base items for P.tune.nb
int64_t bank_matrix_bytes(int prec, const Interp& ip);
// Rebuild the plan's own launches (after a change of its tune config).
void build_plan_schedule(Plan& P, hipStream_t s);
// Launch pairs of the low-rank coupling step of plans with low-rank
// couplings (one plan, or a batch), stage-1 output in T (grown to fit).
std::vector<M2LLaunch> build_aca_schedule(const std::vector<Plan*>& plans,
                                          const TuneConfig& cfg, DevBuf<float>& T,
                                          int64_t T_budget, int64_t* tally, hipStream_t s);
// The library's static workspace (noalloc.hip): its size, and its address
// on the current device (looked up once per device).
int64_t static_workspace_bytes();
void* static_workspace();
// Bytes of the streamed-bank workspace a plan's schedule uses (0: resident).
int64_t plan_workspace_bytes(const Plan& P);
// (Re)create the per-launch timing events of the plan's schedule.
void plan_launch_events(Plan& P);
// A bank range [b0, b1) of one plan in a coupling launch.
struct SchedSource {
  Plan* P;
  int64_t b0, b1;
};
// Launches covering every coupling item of `plans` once (and their near
// field when cfg.p2p_in_queue): resident banks in one launch; streamed
// banks packed into launches of at most ws_matrices generated matrices.
std::vector<M2LLaunch> build_schedule(const std::vector<Plan*>& plans, const TuneConfig& cfg,
                                      void* ws, int64_t ws_matrices, hipStream_t s);
// done: optional events recorded after each launch (one per launch).
void run_schedule(std::vector<M2LLaunch>& sched, int32_t* heads, int prec, const Interp& ip,
                  const TuneConfig& cfg, hipStream_t s, hipEvent_t* done = nullptr);

// coupling kernels (m2l.hip)
void launch_bank_matrices(const M2LLaunch& L, int prec, const Interp& ip, hipStream_t s);
void launch_bank_direct(const int32_t* info, int64_t n_mat, const BankLevel* lv, int prec,
                        const Interp& ip, void* dst, hipStream_t s);
void launch_m2l_items(const M2LLaunch& L, int prec, int Kp, const TuneConfig& cfg,
                      int32_t* head, hipStream_t s);
void launch_valid_offsets(const M2LItem* items, int64_t n_items, const int32_t* cand_begin,
                          const int32_t* cand_count, const int32_t* cand, const M2LDesc* descs,
                          const int32_t* tgt_list, const int4* offtab, int pass,
                          int32_t* counts, const int32_t* out_begin, int32_t* out,
                          unsigned long long* blocks_per_off, int32_t* tiles,
                          hipStream_t s);
int m2l_threads(int Kp);
int m2l_row_blocks(int Kp);
// Near-field items can share the coupling launch (FP32 / BF16, Kp <= 256);
// otherwise the near field runs as its own launch whatever the tune says.
inline bool p2p_queue_supported(int prec, int Kp) {
  return prec != FDM_PREC_FP64 && Kp <= 256;
}
// Compacted coupling items exist in the FP32 and BF16 split kernels with 64
// targets per item.
inline bool compact_supported(int prec, int nb) {
  return (prec == FDM_PREC_FP32 || prec == FDM_PREC_BF16X3 || prec == FDM_PREC_BF16X6) &&
         nb == 64;
}
// Matrix-core columns of one coupling step under cfg (zero padding included).
int64_t issued_columns(const Plan& P, const TuneConfig& cfg);
int64_t m2l_resident_groups(int prec, int nb, int Kp, bool parts);
// per-precision coupling launches (m2l_f64.hip, m2l_f32.hip, m2l_bf16.hip)
void launch_items_f64(const M2LLaunch& L, int Kp, int nb, bool persistent, int32_t* head,
                      hipStream_t s);
void launch_items_f32(const M2LLaunch& L, int Kp, int nb, bool persistent, int32_t* head,
                      hipStream_t s);
void launch_items_bf16(const M2LLaunch& L, int Kp, int nb, bool persistent, int32_t* head,
                       hipStream_t s);
void launch_items_bf16x6(const M2LLaunch& L, int Kp, int nb, bool persistent, int32_t* head,
                         hipStream_t s);
int64_t resident_f64(int nb, int Kp, bool parts);
int64_t resident_f32(int nb, int Kp, bool parts);
int64_t resident_bf16(int nb, int Kp, bool parts);
int64_t resident_bf16x6(int nb, int Kp, bool parts);
// low-rank couplings (aca.hip, m2l_aca.hip)
int64_t aca_matrix_bytes(const Interp& ip, int kp);
void launch_aca(const int32_t* info, int64_t n_mat, const BankLevel* lv, const Interp& ip,
                double eps, int kp, float* bank, int32_t* rank, hipStream_t s);
void launch_items_aca(const M2LLaunch& L, int stage, int Kp, bool persistent, int32_t* head,
                      hipStream_t s);
int64_t resident_aca(int stage, int Kp);

// launch-shape helpers of the C ABI (plan.hip)
TuneConfig check_tune(const fdm_tune& t);
fdm_tune to_c(const TuneConfig& c);
void apply_plan_tune(Plan& P, const TuneConfig& c, hipStream_t s);

}  // namespace fdm

// The opaque handles of the C ABI.
struct fdm_plan {
  fdm::Plan p;
};

struct fdm_batch {
  std::vector<fdm::Plan*> plans;
  int prec = 0;
  fdm::Interp ip;
  fdm::TuneConfig tune;
  int64_t ws_bytes = 0;
  fdm::DevBuf<uint8_t> ws;
  std::vector<fdm::M2LLaunch> sched;
  fdm::DevBuf<int32_t> heads;
  // graph of the whole batched matvec, for the pointers it was captured with
  hipGraphExec_t graph = nullptr;
  std::vector<const void*> graph_v;
  std::vector<void*> graph_y;
  hipStream_t graph_stream = nullptr;
  int graph_c64 = -1;
  bool use_graph = true;
  int aca_kp = 0;                // low-rank couplings (all plans), else 0
  fdm::DevBuf<float> aca_T;      // their stage-1 output
  int64_t tally = 0;
};
