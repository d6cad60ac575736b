// Host tables of the block partition and of the directions.
//
// Admissibility (Sect. 2.2, Def. of directional admissibility): (A1)
// max diam <= eta2 dist and (A3) kappa max diam^2 <= eta2 dist, compared in
// squared form in FP64 with equality admissible.  For two boxes of one
// level with integer offset o the gap along axis d is max(|o_d| - 1, 0) h.
//
// Block tree (Sect. 2.3, Alg. 2) on trees refined to a fixed depth: a pair
// on level l is a block iff its parent pair was refined, i.e. the parent
// offset ceil((o - q)/2) (q the target's octant) was inadmissible -- an
// admissible parent makes every child admissible, so one level of history
// suffices.  Admissible pairs are couplings; inadmissible pairs on the leaf
// level are near-field blocks.
//
// Directions (Sect. 2.4, Alg. 3 and the dir maps): 6 * 4^(l_hf - l) faces per
// level; face index = face * n^2 + quadtree index of the sub-face, faces
// ordered {x=-1},{x=+1},{y=-1},{y=+1},{z=-1},{z=+1}, sub-face coordinates
// measured along sign(face) e_b, lower free axis the more significant bit,
// closed faces with ties to the lowest index.  Between cubic boxes the
// direction argument is the integer offset, so the map is evaluated exactly.
#include <algorithm>
#include <cmath>
#include <set>

#include "plan.hpp"

namespace fdm {

#pragma clang fp contract(off)

static bool admissible(double kappa, const double h[3], const Off& o, double eta2) {
  double g0 = std::max(std::abs(o.x) - 1, 0);
  double g1 = std::max(std::abs(o.y) - 1, 0);
  double g2 = std::max(std::abs(o.z) - 1, 0);
  double d2 = h[0] * h[0] + h[1] * h[1] + h[2] * h[2];
  double s2 = (g0 * h[0]) * (g0 * h[0]) + (g1 * h[1]) * (g1 * h[1]) + (g2 * h[2]) * (g2 * h[2]);
  double e2 = eta2 * eta2;
  bool a1 = d2 <= e2 * s2;
  bool a3 = (kappa * kappa) * (d2 * d2) <= e2 * s2;
  return a1 && a3;
}

static int ceil_half(int v) { return (v + 1) >> 1; }  // ceil(v / 2), arithmetic shift

std::vector<LevelTable> build_level_tables(double kappa, const double side[3], int levels,
                                           int l_hf, double eta2) {
  std::vector<LevelTable> tab(levels + 1);
  tab[0].inadm.push_back({0, 0, 0});  // the root pair: offset 0, never admissible
  int64_t scale[3];
  side_scale(side, scale);
  for (int l = 1; l <= levels; ++l) {
    const double h[3] = {side[0] * std::ldexp(1.0, -l), side[1] * std::ldexp(1.0, -l),
                         side[2] * std::ldexp(1.0, -l)};
    const int lim = (1 << l) - 1;
    std::set<Off> parents(tab[l - 1].inadm.begin(), tab[l - 1].inadm.end());
    std::set<Off> cand;
    for (const Off& O : tab[l - 1].inadm)
      for (int dx = -1; dx <= 1; ++dx)
        for (int dy = -1; dy <= 1; ++dy)
          for (int dz = -1; dz <= 1; ++dz) {
            Off o{2 * O.x + dx, 2 * O.y + dy, 2 * O.z + dz};
            if (std::abs(o.x) <= lim && std::abs(o.y) <= lim && std::abs(o.z) <= lim)
              cand.insert(o);
          }
    LevelTable& T = tab[l];
    for (const Off& o : cand) {
      if (admissible(kappa, h, o, eta2)) {
        uint8_t mask = 0;
        for (int q = 0; q < 8; ++q) {
          Off P{ceil_half(o.x - ((q >> 2) & 1)), ceil_half(o.y - ((q >> 1) & 1)),
                ceil_half(o.z - (q & 1))};
          if (parents.count(P)) mask |= uint8_t(1u << q);
        }
        T.adm.push_back(o);
        T.mask.push_back(mask);
        T.dir.push_back(direction_index(l, l_hf, o, scale));
      } else {
        T.inadm.push_back(o);
      }
    }
  }
  return tab;
}

int direction_count(int level, int l_hf) {
  if (level > l_hf) return 1;
  return 6 * (1 << (2 * (l_hf - level)));
}

void side_scale(const double side[3], int64_t scale[3]) {
  if (side[0] == side[1] && side[1] == side[2]) {
    scale[0] = scale[1] = scale[2] = 1;
    return;
  }
  // side_d = mant_d 2^exp_d with odd integer mantissas; then shift to the
  // smallest exponent
  int64_t mant[3];
  int ex[3];
  for (int d = 0; d < 3; ++d) {
    int e = 0;
    const double f = std::frexp(side[d], &e);
    int64_t m = static_cast<int64_t>(std::ldexp(f, 53));
    e -= 53;
    while (m % 2 == 0) {
      m /= 2;
      ++e;
    }
    mant[d] = m;
    ex[d] = e;
  }
  const int emin = std::min(ex[0], std::min(ex[1], ex[2]));
  for (int d = 0; d < 3; ++d) {
    const int sh = ex[d] - emin;
    if (sh > 62 || (sh > 0 && mant[d] > (INT64_MAX >> sh)))
      fail(FDM_ERR_UNSUPPORTED, "root box sides too unequal for the exact direction map");
    scale[d] = mant[d] << sh;
  }
}

int direction_index(int level, int l_hf, const Off& o) {
  const int64_t one[3] = {1, 1, 1};
  return direction_index(level, l_hf, o, one);
}

int direction_index(int level, int l_hf, const Off& o, const int64_t scale[3]) {
  if (level > l_hf) return 0;
  // the centre offset o * h up to a positive factor, exactly (|o| < 2^10,
  // scale < 2^63: products < 2^73, later terms < 2^83)
  const __int128 v[3] = {__int128(o.x) * scale[0], __int128(o.y) * scale[1],
                         __int128(o.z) * scale[2]};
  auto mag = [](__int128 x) { return x < 0 ? -x : x; };
  const __int128 M = std::max(mag(v[0]), std::max(mag(v[1]), mag(v[2])));
  if (M == 0) return -1;
  int a = 0;
  while (mag(v[a]) != M) ++a;  // lowest axis attaining the maximum
  const int sgn = v[a] > 0 ? 1 : -1;
  const int64_t n = int64_t(1) << (l_hf - level);
  int64_t idx[2];
  int j = 0;
  for (int b = 0; b < 3; ++b) {
    if (b == a) continue;
    const __int128 num = (sgn * v[b] + M) * n;  // >= 0
    const __int128 den = 2 * M;
    const __int128 i = (num + den - 1) / den - 1;  // closed cells, lowest index
    idx[j++] = i < 0 ? 0 : static_cast<int64_t>(i);
  }
  int64_t q = 0;
  for (int bit = l_hf - level - 1; bit >= 0; --bit)
    q = q * 4 + 2 * ((idx[0] >> bit) & 1) + ((idx[1] >> bit) & 1);
  const int face = 2 * a + (sgn > 0 ? 1 : 0);
  return static_cast<int>(face * n * n + q);
}

std::vector<double> direction_vectors(int level, int l_hf) {
  const int nd = direction_count(level, l_hf);
  std::vector<double> out(3 * nd, 0.0);
  if (level > l_hf) return out;  // the single direction 0
  const int k = l_hf - level;
  const int64_t n = int64_t(1) << k;
  for (int jd = 0; jd < nd; ++jd) {
    const int face = static_cast<int>(jd / (n * n));
    int64_t q = jd % (n * n);
    int64_t i1 = 0, i2 = 0;
    for (int bit = 0; bit < k; ++bit) {
      i2 |= ((q >> (2 * bit)) & 1) << bit;
      i1 |= ((q >> (2 * bit + 1)) & 1) << bit;
    }
    const int a = face / 2;
    const double sgn = (face % 2) ? 1.0 : -1.0;
    double vec[3];
    vec[a] = sgn;
    int j = 0;
    for (int b = 0; b < 3; ++b) {
      if (b == a) continue;
      const int64_t i = j == 0 ? i1 : i2;
      vec[b] = sgn * (-1.0 + double(2 * i + 1) / double(n));
      ++j;
    }
    const double nrm = std::sqrt(vec[0] * vec[0] + vec[1] * vec[1] + vec[2] * vec[2]);
    for (int d = 0; d < 3; ++d) out[3 * jd + d] = vec[d] / nrm;
  }
  return out;
}

}  // namespace fdm
