/*
 * fdm.h -- C ABI of the MI355X (gfx950) fast directional Helmholtz matvec.
 *
 * The library computes y ~= A v for the dense matrix
 *
 *     A[j,k] = f(x_j, y_k),   f(x,y) = exp(i kappa |x-y|) / (4 pi |x-y|)
 *
 * (Of & Watschinger, "Complexity Analysis of a Fast Directional Matrix-Vector
 * Multiplication", Sect. 1, eq. of the Helmholtz matrix), for target points
 * x_j and source points y_k in R^3, by the fast directional method of the
 * same paper: uniform box cluster trees (Sect. 2.1, Alg. 1), the directional
 * block partition (Sect. 2.2 admissibility (A1)/(A3), Sect. 2.3 Alg. 2),
 * direction sets (Sect. 2.4 Alg. 3), directional tensor Chebyshev
 * interpolation with nested transfers (Sect. 2.2, 2.5, 2.7), applied by
 * Alg. 4 (Sect. 2.6).  f(x,x) = 0 for bitwise-equal points (the zeroed
 * diagonal of Sect. 4).
 *
 * Conventions shared by every entry point:
 *  - Every function returns an int status: FDM_OK (0) or a negative
 *    fdm_status.  On error nothing is allocated or left behind, *out
 *    pointers are set to NULL, and fdm_last_error() holds a message
 *    (thread-local; valid until the next call on the same thread).
 *  - "device" pointers are HIP device memory of the current device;
 *    "host" pointers are ordinary host memory.
 *  - stream: a hipStream_t passed as void* (NULL = the null stream).  All
 *    device work of a call is enqueued on it.
 *  - Complex numbers are interleaved (re, im) pairs: complex128 = two
 *    doubles, complex64 = two floats.
 *  - Points are n x 3 row-major FP64 arrays (x, y, z per point).
 */
#ifndef FDM_H
#define FDM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fdm_plan fdm_plan;

/* Precision of the coupling (M2L) step; every other step runs in FP64. */
typedef enum {
  FDM_PREC_FP64 = 0,   /* plain: FP64 matrix-core products, FP64 sums      */
  FDM_PREC_FP32 = 1,   /* mixed: FP32 operands and matrix-core accumulation */
  FDM_PREC_BF16X3 = 2, /* mixed: BF16 hi/lo split, 3 products, FP32 sums   */
  FDM_PREC_BF16X6 = 3  /* mixed: BF16 hi/mid/lo split of FP64 operands, the
                          6 part products of order <= 2, FP32 sums        */
} fdm_precision;

typedef enum {
  FDM_OK = 0,
  FDM_ERR_INVALID_ARG = -1,
  FDM_ERR_POINT_OUTSIDE_BOX = -2,
  FDM_ERR_UNSUPPORTED = -3,
  FDM_ERR_OUT_OF_MEMORY = -4,
  FDM_ERR_HIP = -5,
  FDM_ERR_STATE = -6
} fdm_status;

/*
 * fdm_build_tree -- build a plan: both uniform box cluster trees (Alg. 1,
 * refined to a fixed depth), the block partition (Alg. 2 with (A1)/(A3),
 * eta2 = 5), the direction sets (Alg. 3) and the coupling-matrix bank (one
 * matrix per level and offset, Sect. 2.7).
 *
 *  points_T  device, n_T x 3 FP64 target points (user order); read only
 *            during the call.
 *  points_S  device, n_S x 3 FP64 source points (user order); read only
 *            during the call.  May equal points_T.
 *  kappa     wave number, finite, >= 0 (0 gives the Laplace kernel).
 *  box       host, 6 doubles {lo_x, lo_y, lo_z, hi_x, hi_y, hi_z}: the root
 *            box (lo, hi] shared by both trees, any axis-parallel box
 *            (Sect. 2.1): the boxes of a level are its translates scaled by
 *            2^-level per axis, and the direction of a box pair is that of
 *            its centre offset, evaluated exactly (FDM_ERR_UNSUPPORTED only
 *            for sides whose binary mantissas and exponents do not fit one
 *            63-bit integer scale); the high-frequency rule uses the longest
 *            side.  Every point must satisfy lo < x <= hi per axis (else
 *            FDM_ERR_POINT_OUTSIDE_BOX).
 *  levels    tree depth below the root, 0..9 (the per-level key -> box
 *            grids hold 8^levels entries); every non-empty box above this
 *            level is split (leaves all sit on this level).  levels outside
 *            0..9 give FDM_ERR_INVALID_ARG.
 *  m         Chebyshev degree per axis: (m+1)^3 nodes per box.  m outside
 *            1..8 gives FDM_ERR_INVALID_ARG.  The coupling kernels give one
 *            wave to each 32 of the (m+1)^3 nodes padded to a multiple of
 *            32, at most 384 rows per workgroup: at m = 7 and 8 (512 and
 *            736 padded rows) each coupling item runs once per row block.
 *            Low-rank couplings (aca_eps > 0) need m <= 6
 *            (FDM_ERR_UNSUPPORTED).
 *  precision an fdm_precision.
 *  stream    HIP stream for the device work; the call synchronises it
 *            before returning (box counts size the plan).
 *  out       receives the plan (owned by the caller; free with
 *            fdm_plan_destroy).  The plan owns device copies of everything
 *            it needs, so the point buffers may be freed after the call.
 *
 * The high-frequency level l_hf is the largest level l <= levels with
 * kappa * h_l >= 3.2 (h_l the box side), else -1.
 */
int fdm_build_tree(const double* points_T, int64_t n_T,
                   const double* points_S, int64_t n_S,
                   double kappa, const double box[6], int levels, int m,
                   int precision, void* stream, fdm_plan** out);

/* fdm_build_tree with explicit l_hf (-1 .. levels; -2 = automatic rule). */
int fdm_build_tree_ex(const double* points_T, int64_t n_T,
                      const double* points_S, int64_t n_S,
                      double kappa, const double box[6], int levels, int m,
                      int precision, int l_hf, void* stream, fdm_plan** out);

/*
 * Launch shape of the coupling step (Sect. 2.6, M2L) and near field.
 *  nb            target boxes per coupling work item: 32 or 64.
 *  persistent    1: one workgroup per compute-unit slot, each pulling work
 *                items from a device queue until it is empty; 0: one
 *                workgroup per item.
 *  lpt           1: items with the most offsets first; 0: items in (level,
 *                octant, direction, target block) order.
 *  p2p_in_queue  1: the near-field work (blocks of target points) is queued
 *                behind the coupling items of the same launch; 0: separate
 *                launch.
 *  compact       column compaction of the mixed FP32 and BF16 split
 *                coupling items (nb 64): per offset only the target boxes
 *                whose source box is non-empty take matrix-core columns.
 *                0: never; 1: on levels where it saves at least a fifth of
 *                the columns (sparse leaf levels); 2: on every level.  No
 *                effect in plain FP64.
 * Results do not depend on the launch shape except through nb, which
 * changes the grouping of the FP32 partial sums (the FP64 path is summed in
 * the same order for both nb); compaction skips zero columns only and
 * leaves every partial sum and flush point as it is.  A zero
 * fdm_options.tune.nb selects the defaults {64, 1, 1, 0, 1}, or {32, 1, 1, 0,
 * 1} for FDM_PREC_BF16X6, whose 64-target items need more registers than a
 * workgroup of 11 or 12 waves leaves them (their spills make them slower
 * than 32-target items; compaction needs 64-target items and is then off).
 */
typedef struct {
  int32_t nb;
  int32_t persistent;
  int32_t lpt;
  int32_t p2p_in_queue;
  int32_t compact;
} fdm_tune;

/*
 * Plan options.
 *  precision          an fdm_precision.
 *  l_hf               -2 = the automatic rule of fdm_build_tree, else
 *                     -1 .. levels.
 *  bank_budget_bytes  0: the coupling bank (one matrix per level and
 *                     offset, Sect. 2.7) is generated once and held by the
 *                     plan.  > 0: the plan holds no bank; each matvec
 *                     generates it, a range of matrices at a time, into a
 *                     workspace of at most this many bytes (at least one
 *                     matrix), allocated at the plan's first matvec.  Use it
 *                     when the bank does not fit, and for plans that only run
 *                     in a batch (which brings its own workspace).
 *  tune               initial launch shape (NULL-equivalent: nb = 0 picks
 *                     the defaults {64, 1, 1, 0, 1}).
 *  full_bank          0: a resident FP64 or FP32 bank stores one matrix per
 *                     pair of offsets (o, -o) and applies the matrix of -o
 *                     as the transpose of that of o (A_{-o} = A_o^T: the
 *                     coupling function is symmetric and the direction map
 *                     odd), halving the bank; 1: one matrix per offset.
 *                     Streamed and BF16 split banks always hold one matrix
 *                     per offset.  Results agree to rounding (the k sums of
 *                     transposed matrices run in another order).
 *  aca_eps            > 0: low-rank couplings (Sect. 2.7).  At plan build
 *                     every stored coupling matrix is compressed on the device
 *                     by partially pivoted adaptive cross approximation
 *                     (the pivot rule and stopping test of fdm_aca, tolerance
 *                     aca_eps, at most aca_rank crosses), A ~ U Vt, and each
 *                     matvec applies it in two matrix-core stages, T = Vt v
 *                     then U T (16 K k instead of 8 K^2 flops per block).
 *                     FDM_PREC_FP32 only (else FDM_ERR_UNSUPPORTED), resident
 *                     bank only (bank_budget_bytes 0, else
 *                     FDM_ERR_INVALID_ARG); launch shape fixed to 64 targets
 *                     per item, no compaction, near field apart.  0: dense
 *                     couplings.  Must be finite and >= 0.
 *  aca_rank           rank cap of the low-rank couplings: 32 or 64 (0: 64);
 *                     a matrix that needs more crosses keeps the first
 *                     aca_rank (fdm_plan_stats reports the largest rank).
 *  aca_chunk_bytes    low-rank couplings: bound on the first stage's output
 *                     held at once.  Each item's offsets are ordered by rank
 *                     and cut into groups of 16 (each run at its padded
 *                     rank); a launch pair covers one group of as many items
 *                     as fit (at least one).  0: 8 GiB; >= 0.
 *  n_max              Alg. 1's stop rule (Sect. 2.1): a box is refined only
 *                     while it holds more than n_max points (and lies above
 *                     level `levels`), so leaves sit on several levels and
 *                     near-field blocks (a leaf against a box of any size)
 *                     on every level (Alg. 2).  0: every non-empty box is
 *                     refined down to `levels` (a uniform tree).  >= 0 (else
 *                     FDM_ERR_INVALID_ARG); when > 0 the near field never
 *                     shares the coupling queue.
 */
typedef struct {
  int32_t precision;
  int32_t l_hf;
  int64_t bank_budget_bytes;
  fdm_tune tune;
  int32_t full_bank;
  int32_t aca_rank;
  double aca_eps;
  int64_t aca_chunk_bytes;
  int64_t n_max;
} fdm_options;

/* fdm_build_tree with options (opts host, not NULL). */
int fdm_build_tree_opts(const double* points_T, int64_t n_T,
                        const double* points_S, int64_t n_S,
                        double kappa, const double box[6], int levels, int m,
                        const fdm_options* opts, void* stream, fdm_plan** out);

/*
 * Launch shape of a plan: read, or set (rebuilds the plan's work lists when
 * nb changes; synchronises stream).  FDM_ERR_INVALID_ARG for nb not 32/64,
 * flags not 0/1 or compact not 0..2; FDM_ERR_STATE while the plan belongs
 * to a batch.
 */
int fdm_plan_get_tune(const fdm_plan* plan, fdm_tune* out);
int fdm_plan_set_tune(fdm_plan* plan, const fdm_tune* tune, void* stream);

/*
 * fdm_plan_autotune -- time the coupling step under each candidate launch
 * shape (nb in {64, 32} x persistent in {1, 0} x lpt in {1, 0}, near field
 * and compaction kept as set; then, for FP32 and BF16 split plans without
 * low-rank couplings, the two other compaction modes at nb 64, persistent,
 * heaviest first) on the plan's own data and keep the fastest.  Runs one
 * full matvec of v into y first (same arguments as
 * fdm_plan_matvec{,_c64}), then one coupling step per candidate, and
 * synchronises stream.
 *  max_candidates  how many of the candidates to try, in the order above
 *                  (1..8, or 1..10 where the compaction modes are added).
 *  best            host, receives the chosen shape (may be NULL).
 *  ms              host array of max_candidates doubles receiving each
 *                  candidate's coupling-step time (may be NULL).
 */
int fdm_plan_autotune(fdm_plan* plan, const void* v, void* y, int c64,
                      int max_candidates, void* stream, fdm_tune* best,
                      double* ms);

/*
 * fdm_plan_matvec -- y = A~ v by Alg. 4 (S2M, M2M, M2L, L2L, L2T, near
 * field), asynchronously on `stream`.
 *
 *  v  device, n_S complex128 (user order of the sources); not modified.
 *  y  device, n_T complex128 (user order of the targets); overwritten.
 *     v and y must not overlap.
 *
 * At most one matvec may be in flight per plan (the plan's workspaces are
 * reused); calls on different plans may overlap.
 */
int fdm_plan_matvec(fdm_plan* plan, const void* v, void* y, void* stream);

/* As fdm_plan_matvec with complex64 v and y (FP64 accumulation inside). */
int fdm_plan_matvec_c64(fdm_plan* plan, const void* v, void* y, void* stream);

/*
 * fdm_plan_matvec_multi -- Y = A~ V for nrhs right-hand sides (repeated
 * application of one operator, Sect. 4): the plan's trees, work lists and
 * coupling bank serve every vector.  On uniform trees whose near field runs
 * apart from the coupling queue, the near field evaluates each kernel value
 * once for up to four vectors; otherwise (adaptive trees, near field queued)
 * it runs vector by vector.  Each result equals fdm_plan_matvec's on the
 * same vector bit for bit.  Asynchronous on `stream`.
 *
 *  V     device, nrhs vectors of n_S complex values one after the other
 *        (complex64 when c64 = 1, else complex128); not modified.
 *  Y     device, nrhs vectors of n_T complex values, same type; overwritten.
 *        V and Y must not overlap.
 *  nrhs  >= 1.  The plan holds two tree-order copies of nrhs vectors
 *        (allocated on the first call with that many, kept for later calls).
 * FDM_ERR_INVALID_ARG for NULL or host pointers, nrhs < 1, c64 not 0/1, or
 * overlapping V and Y; FDM_ERR_STATE while the plan belongs to a batch.
 */
int fdm_plan_matvec_multi(fdm_plan* plan, const void* V, void* Y, int nrhs, int c64,
                          void* stream);

/*
 * Per-phase timing of later matvecs with HIP events recorded on the matvec's
 * stream (enable != 0 turns it on).  fdm_plan_phase_ms waits for the last
 * matvec's events and writes 7 values in milliseconds: S2M, M2M, M2L, L2L,
 * L2T, near field, whole matvec.  FDM_ERR_STATE if timing is off or no
 * matvec ran since it was enabled.
 */
int fdm_plan_set_timing(fdm_plan* plan, int enable);
int fdm_plan_phase_ms(const fdm_plan* plan, double ms[7]);

/*
 * fdm_plan_prepare -- build now what the plan's first matvec would build:
 * its coupling launch schedule and, for a streamed bank, the workspace
 * (synchronises stream).  Matvecs after it allocate nothing.
 */
int fdm_plan_prepare(fdm_plan* plan, void* stream);

/*
 * Progress of a long matvec: the number of coupling launches of the plan's
 * schedule (FDM_ERR_STATE before fdm_plan_prepare or the first matvec), and,
 * with timing on, a wait for launch i (0-based) of the last timed matvec,
 * returning the milliseconds from the matvec's start to that launch's end.
 */
int fdm_plan_coupling_launches(const fdm_plan* plan, int* n);
int fdm_plan_wait_launch(const fdm_plan* plan, int i, double* ms);

/*
 * fdm_plan_matvec_noalloc -- fdm_plan_matvec (c64 = 0) or
 * fdm_plan_matvec_c64 (c64 = 1) that allocates no memory, for callers that
 * cannot allocate: code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc.  For plans with a streamed coupling bank
 * (bank_budget_bytes > 0), whose matvec otherwise generates the bank into a
 * workspace the plan allocates: here the bank goes to a static workspace of
 * the library, 64 MiB on each GPU, held until the process ends.
 *
 *  plan    built with 0 < bank_budget_bytes and a bank workspace of at most
 *          64 MiB (the workspace holds min(N_SC, floor(budget / matrix))
 *          coupling matrices), else FDM_ERR_INVALID_ARG; prepared with
 *          fdm_plan_prepare (which builds the launch schedule for the static
 *          workspace), else FDM_ERR_STATE.
 *  v, y    as for fdm_plan_matvec / fdm_plan_matvec_c64.
 * Results are bit for bit those of fdm_plan_matvec{,_c64} on the same plan.
 * Every such call on one GPU shares that GPU's static workspace: calls that
 * overlap on one GPU (other streams, other threads, other plans) race and
 * must be serialised by the caller.  Nothing in the workspace needs to start
 * at zero.  No hipMalloc, hipFree or allocating library call is made.
 */
int fdm_plan_matvec_noalloc(fdm_plan* plan, const void* v, void* y, int c64,
                            void* stream);

/* Free a plan and all its device memory.  NULL is accepted. */
int fdm_plan_destroy(fdm_plan* plan);

/* Plan statistics (Table 1 of Sect. 4 lists N_C, N_SC and nf). */
typedef struct {
  int64_t n_T, n_S;
  int32_t levels, m, K, precision;
  int32_t l_hf, l_min;          /* l_min: coarsest level with a coupling */
  int64_t n_couplings;          /* N_C: admissible blocks                  */
  int64_t n_stored_couplings;   /* N_SC: distinct (level, offset) used     */
  int64_t n_bank_matrices;      /* coupling matrices in the resident bank
                                   (one per admissible offset, or one per
                                   pair (o, -o), see full_bank), or, for a
                                   streamed bank, generated per matvec     */
  int64_t near_pairs;           /* inadmissible leaf blocks                */
  int64_t near_entries;         /* sum of #t * #s over inadmissible blocks  */
  int64_t m2l_columns;          /* coupling products issued by the M2L
                                   kernel under the plan's launch shape,
                                   incl. zero-padded columns                */
  int64_t device_bytes;         /* device memory held by the plan          */
  double setup_ms;              /* wall time of fdm_build_tree             */
  int32_t aca_rank_cap;         /* low-rank couplings: rank cap, else 0    */
  int32_t aca_rank_max;         /* largest rank among the stored matrices  */
  double aca_rank_mean;         /* mean rank                               */
  double aca_flops;             /* low-rank coupling step: real flops of the
                                   two products over the admissible blocks,
                                   16 K r per block at its matrix's rank r */
  double aca_issued_flops;      /* what its kernels issue: padded ranks,
                                   rows to Kp, 64 target slots per item    */
} fdm_stats;

int fdm_plan_stats(const fdm_plan* plan, fdm_stats* out);

/*
 * fdm_plan_export -- copy a named plan array to host memory (structure
 * parity and debugging).  Query the size with host == NULL.
 *
 *  name   one of (l a decimal level, X = T or S):
 *           "perm_X"      int64[n]   tree slot -> user index
 *           "keys_Xl"     int64[nb]  Morton keys of the boxes on level l
 *           "start_Xl"    int64[nb]  first tree slot of each box
 *           "count_Xl"    int64[nb]  number of points of each box
 *           "l_hf"        int64[1]
 *           "nc_l"        int64[1]   admissible blocks on level l
 *           "off_l"       int64[3n]  distinct offsets of those blocks,
 *                                    sorted lexicographically
 *           "offdir_l"    int64[n]   direction index of each offset
 *           "offcnt_l"    int64[n]   number of blocks using each offset
 *           "dirs_l"      double[3 nd] direction vectors of level l
 *           "D_Xl", "Dh_Xl" int64[]  active / inherited directions,
 *                                    sorted codes box * nd + dir
 *           "near_pairs", "near_entries"  int64[1]
 *           "aca_rank"    int64[n]   low-rank couplings: crosses taken per
 *                                    stored matrix (bank id order)
 *           "bank_offsets" int64[5n] per bank id: level, offset x, y, z and
 *                                    direction index of its matrix
 *           "mom_l", "loc_l"  complex128[nb * nd * K] moments / locals of
 *                                    the last matvec (centre-relative
 *                                    phase form, box-major)
 *  host   destination or NULL; capacity its size in bytes.
 *  size   receives the size in bytes.
 * Unknown names give FDM_ERR_INVALID_ARG; a short capacity gives
 * FDM_ERR_INVALID_ARG with *size set.
 */
int fdm_plan_export(const fdm_plan* plan, const char* name, void* host,
                    int64_t capacity, int64_t* size);

/*
 * fdm_dense_matvec -- the dense product y = A v by direct summation in
 * FP64 on the GPU (Sect. 1), for reference and timing.
 *  points_T/points_S device n x 3 FP64; v device complex128[n_S];
 *  y device complex128[n_T], overwritten.  Asynchronous on stream.
 */
int fdm_dense_matvec(const double* points_T, int64_t n_T,
                     const double* points_S, int64_t n_S, double kappa,
                     const void* v, void* y, void* stream);

/*
 * Batched matvecs (many independent problems, possibly of different sizes
 * and wave numbers, one launch sequence).
 *
 * fdm_batch_create -- group n plans (same m and precision, each in at most
 * one batch; with low-rank couplings either all, with one rank cap, or none,
 * else FDM_ERR_UNSUPPORTED) into a batch.  The plans stay owned by the
 * caller and must
 * outlive the batch; while they belong to it they cannot be re-tuned or
 * destroyed (FDM_ERR_STATE).  Plans built with bank_budget_bytes > 0 have
 * their coupling banks generated during each batched matvec into one
 * workspace owned by the batch, of workspace_bytes (0: the smaller of what
 * all such banks need and half of the free device memory), at least one
 * matrix; plans with resident banks use them.
 *  plans   host array of n plan handles.
 *  stream  used for the set-up uploads; synchronised.
 *
 * Each batched matvec runs: for every plan the permutation and forward
 * transformation (S2M, M2M); then the coupling step of all plans as
 * persistent launches pulling from one device queue over (plan, level,
 * direction, target block) items, with every plan's near field queued
 * behind them (one launch when all banks are resident or fit the
 * workspace; low-rank plans: launch pairs over every plan's offset groups,
 * near field apart); then for every plan L2L, L2T and the permutation back.
 */
typedef struct fdm_batch fdm_batch;

int fdm_batch_create(fdm_plan* const* plans, int n, int64_t workspace_bytes,
                     void* stream, fdm_batch** out);

/*
 * fdm_batch_matvec -- y_i = A~_i v_i for every plan i of the batch.
 *  v  host array of n device pointers: complex128[n_S(i)], or complex64
 *     when c64 != 0.
 *  y  host array of n device pointers: complex128[n_T(i)] (complex64 when
 *     c64 != 0), overwritten.  No y may overlap any v or another y.
 * Asynchronous on stream.  With graphs enabled (the default) and a
 * non-NULL stream, the whole batched matvec is captured once into a HIP
 * graph for these pointers and stream and replayed on later calls with the
 * same pointers; other pointers re-capture.  Not re-entrant per batch.
 */
int fdm_batch_matvec(fdm_batch* batch, const void* const* v, void* const* y,
                     int c64, void* stream);

/* Enable (1) or disable (0) graph capture of batched matvecs. */
int fdm_batch_set_graph(fdm_batch* batch, int enable);

/* Launch shape of the batch's coupling launches (as for plans; rebuilds the
 * work lists of its plans when nb changes; synchronises stream). */
int fdm_batch_get_tune(const fdm_batch* batch, fdm_tune* out);
int fdm_batch_set_tune(fdm_batch* batch, const fdm_tune* tune, void* stream);

/*
 * fdm_batch_autotune -- as fdm_plan_autotune for the batch's coupling
 * launches: one batched matvec, then one timed coupling step per candidate
 * (nb in {64, 32} x lpt in {1, 0}; persistent launches with the near field
 * queued; then, as for a plan, the two other compaction modes: 1..4, or
 * 1..6 candidates), keeping the fastest.
 */
int fdm_batch_autotune(fdm_batch* batch, const void* const* v, void* const* y,
                       int c64, int max_candidates, void* stream,
                       fdm_tune* best, double* ms);

/* Free a batch (not its plans).  NULL is accepted. */
int fdm_batch_destroy(fdm_batch* batch);

/*
 * fdm_aca -- low-rank compression A ~ U W^H of one complex matrix by
 * partially pivoted adaptive cross approximation, the compression the paper
 * applies to its coupling matrices (Sect. 2.7).  Cross k takes the residual
 * of one row of A, scales it by its entry of largest modulus (the pivot
 * column), takes the residual of that column, and moves on to the unused row
 * where that column is largest; a row whose residual vanishes is skipped for
 * the first unused row.  It stops once |u_k| |v_k| <= eps |sum_l u_l v_l^T|_F
 * (the Frobenius norm kept up to date from inner products), at max_rank
 * crosses, or when no unused row is left.  Only the pivot rows and columns
 * of A are read.
 * Host code: runs on the calling thread, touches no device and no stream.
 *  A        host complex128 (re, im interleaved), n_rows x n_cols, row-major.
 *  eps      relative tolerance, >= 0 (0: stop only at max_rank or when the
 *           residual of every row has vanished).
 *  max_rank 1..min(n_rows, n_cols).
 *  U        host complex128, n_rows x max_rank, row-major: column l holds u_l
 *           for l < *rank; the other columns are zeroed.
 *  W        host complex128, n_cols x max_rank, row-major: column l holds
 *           conj(v_l), so that A ~ U W^H.  Same zeroing.
 *  rank     host int, set to the number of crosses taken (0 for A = 0).
 * U and W are owned by the caller and may not overlap A or each other.
 * FDM_ERR_INVALID_ARG for NULL pointers, n_rows or n_cols < 1, a max_rank
 * outside the range, a negative or non-finite eps, or non-finite entries in
 * a row or column it reads.
 */
int fdm_aca(const double* A, int n_rows, int n_cols, double eps, int max_rank,
            double* U, double* W, int* rank);

/* Thread-local message of the last error ("" if none). */
const char* fdm_last_error(void);

/* Library version string. */
const char* fdm_version(void);

#ifdef __cplusplus
}
#endif
#endif /* FDM_H */
