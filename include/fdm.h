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
  FDM_PREC_BF16X3 = 2  /* mixed: BF16 hi/lo split, 3 products, FP32 sums   */
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
 *            box (lo, hi] shared by both trees.  Must be a cube (else
 *            FDM_ERR_UNSUPPORTED).  Every point must satisfy lo < x <= hi
 *            per axis (else FDM_ERR_POINT_OUTSIDE_BOX).
 *  levels    tree depth below the root, 0..9; every non-empty box above
 *            this level is split (leaves all sit on this level).
 *  m         Chebyshev degree per axis, 1..8: (m+1)^3 nodes per box.
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
 * Per-phase timing of later matvecs with HIP events recorded on the matvec's
 * stream (enable != 0 turns it on).  fdm_plan_phase_ms waits for the last
 * matvec's events and writes 7 values in milliseconds: S2M, M2M, M2L, L2L,
 * L2T, near field, whole matvec.  FDM_ERR_STATE if timing is off or no
 * matvec ran since it was enabled.
 */
int fdm_plan_set_timing(fdm_plan* plan, int enable);
int fdm_plan_phase_ms(const fdm_plan* plan, double ms[7]);

/* Free a plan and all its device memory.  NULL is accepted. */
int fdm_plan_destroy(fdm_plan* plan);

/* Plan statistics (Table 1 of Sect. 4 lists N_C, N_SC and nf). */
typedef struct {
  int64_t n_T, n_S;
  int32_t levels, m, K, precision;
  int32_t l_hf, l_min;          /* l_min: coarsest level with a coupling */
  int64_t n_couplings;          /* N_C: admissible blocks                  */
  int64_t n_stored_couplings;   /* N_SC: distinct (level, offset) used     */
  int64_t n_bank_matrices;      /* matrices held (>= N_SC)                 */
  int64_t near_pairs;           /* inadmissible leaf blocks                */
  int64_t near_entries;         /* sum of #t * #s over inadmissible blocks  */
  int64_t m2l_columns;          /* coupling products issued by the M2L
                                   kernel, incl. zero-padded columns        */
  int64_t device_bytes;         /* device memory held by the plan          */
  double setup_ms;              /* wall time of fdm_build_tree             */
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

/* Thread-local message of the last error ("" if none). */
const char* fdm_last_error(void);

/* Library version string. */
const char* fdm_version(void);

#ifdef __cplusplus
}
#endif
#endif /* FDM_H */
