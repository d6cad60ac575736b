// Low-rank compression of a complex matrix by partially pivoted adaptive
// cross approximation (Sect. 2.7), A ~ sum_l u_l v_l^T with the pivot row of
// each cross scaled to 1 at its pivot column.  Host code only: it runs at
// plan-build time on matrices the caller holds, touches no device.
#include "capi.hpp"

#include <cmath>
#include <complex>
#include <cstring>
#include <vector>

namespace fdm {
namespace {

using cd = std::complex<double>;

// First index of the largest modulus, passing over entries with skip[i]
// (none when skip is null); -1 if every entry is skipped.
int arg_max_abs(const cd* a, int n, const std::vector<char>* skip) {
  int best = -1;
  double bm = -1.0;
  for (int i = 0; i < n; ++i) {
    if (skip && (*skip)[i]) continue;
    const double m = std::abs(a[i]);
    if (m > bm) {
      bm = m;
      best = i;
    }
  }
  return best;
}

double norm2(const cd* a, int n) {
  double s = 0.0;
  for (int i = 0; i < n; ++i) s += std::norm(a[i]);
  return std::sqrt(s);
}

// sum_i conj(a_i) b_i
cd dot_conj(const cd* a, const cd* b, int n) {
  cd s(0.0, 0.0);
  for (int i = 0; i < n; ++i) s += std::conj(a[i]) * b[i];
  return s;
}

void check_finite(const cd* a, int n, const char* what) {
  for (int i = 0; i < n; ++i)
    if (!std::isfinite(a[i].real()) || !std::isfinite(a[i].imag()))
      fail(FDM_ERR_INVALID_ARG, std::string("fdm_aca: non-finite entry in a ") + what);
}

// Crosses are kept as contiguous vectors (u_l of n rows, v_l of m columns);
// returns their number.
int aca(const cd* A, int n, int m, double eps, int max_rank, std::vector<cd>& us,
        std::vector<cd>& vs) {
  us.assign(size_t(max_rank) * n, cd());
  vs.assign(size_t(max_rank) * m, cd());
  std::vector<char> used(n, 0);
  std::vector<cd> r(m), u(n);
  double fro2 = 0.0;  // |sum_l u_l v_l^T|_F^2
  int k = 0, i = 0;
  while (k < max_rank) {
    // residual of row i
    std::memcpy(r.data(), A + size_t(i) * m, sizeof(cd) * m);
    check_finite(r.data(), m, "row");
    for (int l = 0; l < k; ++l) {
      const cd ul = us[size_t(l) * n + i];
      const cd* vl = &vs[size_t(l) * m];
      for (int j = 0; j < m; ++j) r[j] -= ul * vl[j];
    }
    used[i] = 1;
    const int j = arg_max_abs(r.data(), m, nullptr);
    if (r[j] == cd(0.0, 0.0)) {  // the row is already reproduced: next unused row
      int f = 0;
      while (f < n && used[f]) ++f;
      if (f == n) break;
      i = f;
      continue;
    }
    cd* v = &vs[size_t(k) * m];
    for (int q = 0; q < m; ++q) v[q] = r[q] / r[j];
    // residual of column j
    for (int q = 0; q < n; ++q) u[q] = A[size_t(q) * m + j];
    check_finite(u.data(), n, "column");
    for (int l = 0; l < k; ++l) {
      const cd vl = vs[size_t(l) * m + j];
      const cd* ul = &us[size_t(l) * n];
      for (int q = 0; q < n; ++q) u[q] -= vl * ul[q];
    }
    // |S_k|^2 = |S_(k-1)|^2 + 2 Re sum_l <u_l, u><v_l, v> + |u|^2 |v|^2
    double cross = 0.0;
    for (int l = 0; l < k; ++l)
      cross += (dot_conj(&us[size_t(l) * n], u.data(), n) *
                dot_conj(&vs[size_t(l) * m], v, m)).real();
    const double nu = norm2(u.data(), n), nv = norm2(v, m);
    fro2 += 2.0 * cross + (nu * nv) * (nu * nv);
    std::memcpy(&us[size_t(k) * n], u.data(), sizeof(cd) * n);
    ++k;
    if (nu * nv <= eps * std::sqrt(std::max(fro2, 0.0))) break;
    const int next = arg_max_abs(u.data(), n, &used);
    if (next < 0) break;  // every row used
    i = next;
  }
  return k;
}

}  // namespace
}  // namespace fdm

using namespace fdm;

extern "C" int fdm_aca(const double* A, int n_rows, int n_cols, double eps, int max_rank,
                       double* U, double* W, int* rank) {
  return guarded([&] {
    if (!A || !U || !W || !rank) fail(FDM_ERR_INVALID_ARG, "fdm_aca: NULL pointer");
    if (n_rows < 1 || n_cols < 1) fail(FDM_ERR_INVALID_ARG, "fdm_aca: empty matrix");
    if (max_rank < 1 || max_rank > std::min(n_rows, n_cols))
      fail(FDM_ERR_INVALID_ARG, "fdm_aca: max_rank outside 1..min(n_rows, n_cols)");
    if (!(eps >= 0.0) || !std::isfinite(eps))
      fail(FDM_ERR_INVALID_ARG, "fdm_aca: eps must be finite and >= 0");
    std::vector<cd> us, vs;
    const int k = aca(reinterpret_cast<const cd*>(A), n_rows, n_cols, eps, max_rank, us, vs);
    cd* Uo = reinterpret_cast<cd*>(U);
    cd* Wo = reinterpret_cast<cd*>(W);
    for (int q = 0; q < n_rows; ++q)
      for (int l = 0; l < max_rank; ++l)
        Uo[size_t(q) * max_rank + l] = l < k ? us[size_t(l) * n_rows + q] : cd();
    for (int q = 0; q < n_cols; ++q)
      for (int l = 0; l < max_rank; ++l)
        Wo[size_t(q) * max_rank + l] = l < k ? std::conj(vs[size_t(l) * n_cols + q]) : cd();
    *rank = k;
  });
}
