/* Plain C99 client of the library's C ABI (include/fdm.h), built and run by
 * tests/test_c_abi_c.py on a host without a GPU: the header compiles as C,
 * the library links, and the host-only entry points work from C. */
#include <math.h>
#include <stdio.h>
#include <string.h>

#include "fdm.h"

#define NR 9
#define NC 7
#define R 4

int main(void) {
  /* A = x y^H + 2 z w^H (rank 2), complex128 interleaved, row-major */
  double A[NR * NC * 2], U[NR * R * 2], W[NC * R * 2];
  int i, j, l, k = -1;
  for (i = 0; i < NR; ++i)
    for (j = 0; j < NC; ++j) {
      double xr = 1.0 + i, xi = 0.5 * i, yr = 2.0 - 0.3 * j, yi = 0.1 * j;
      double zr = cos(0.7 * i), zi = sin(0.7 * i), wr = 1.0 / (1.0 + j), wi = -0.2;
      /* x conj(y) + 2 z conj(w) */
      A[2 * (i * NC + j)] = xr * yr + xi * yi + 2.0 * (zr * wr + zi * wi);
      A[2 * (i * NC + j) + 1] = xi * yr - xr * yi + 2.0 * (zi * wr - zr * wi);
    }
  if (strncmp(fdm_version(), "fdm-gfx950", 10) != 0) return 10;
  if (fdm_aca(A, NR, NC, 1e-14, R, U, W, &k) != FDM_OK) return 11;
  if (k < 2 || k > 3) return 12;
  {
    double err = 0.0, nrm = 0.0;
    for (i = 0; i < NR; ++i)
      for (j = 0; j < NC; ++j) {
        double sr = 0.0, si = 0.0;
        for (l = 0; l < R; ++l) { /* U[i,l] * conj(W[j,l]) */
          double ur = U[2 * (i * R + l)], ui = U[2 * (i * R + l) + 1];
          double wr = W[2 * (j * R + l)], wi = W[2 * (j * R + l) + 1];
          sr += ur * wr + ui * wi;
          si += ui * wr - ur * wi;
        }
        err += pow(sr - A[2 * (i * NC + j)], 2) + pow(si - A[2 * (i * NC + j) + 1], 2);
        nrm += pow(A[2 * (i * NC + j)], 2) + pow(A[2 * (i * NC + j) + 1], 2);
      }
    if (!(sqrt(err) <= 1e-12 * sqrt(nrm))) return 13;
  }
  if (fdm_aca(A, NR, NC, -1.0, R, U, W, &k) != FDM_ERR_INVALID_ARG) return 14;
  if (fdm_last_error()[0] == '\0') return 15;
  if (fdm_plan_destroy(NULL) != FDM_OK) return 16;
  printf("c abi ok: rank %d\n", k);
  return 0;
}
