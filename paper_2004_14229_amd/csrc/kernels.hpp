// Internal interfaces between the plan (host) and the device kernels.
#pragma once

#include "common.hpp"

namespace fdm {

// ---------------------------------------------------------------- sort.hip
int64_t exclusive_scan(const int32_t* in, int32_t* out, int64_t n, hipStream_t s);
void sort_pairs_stable(DevBuf<uint32_t>& keys, DevBuf<int32_t>& vals, int64_t n,
                       int key_bits, hipStream_t s);

// ---------------------------------------------------------------- tree.hip
// Uniform box cluster tree refined to a fixed depth (Sect. 2.1, Alg. 1).
struct DevTree {
  int64_t n = 0;
  int levels = 0;
  DevBuf<double> x, y, z;       // points in tree order (SoA)
  DevBuf<int32_t> perm;         // tree slot -> user index
  DevBuf<int32_t> leaf_of;      // tree slot -> leaf box index
  std::vector<int64_t> nb;      // boxes per level
  std::vector<DevBuf<uint32_t>> key;    // per level: Morton keys (ascending)
  std::vector<DevBuf<int32_t>> start;   // per level: first tree slot
  std::vector<DevBuf<int32_t>> count;   // per level: number of points
  std::vector<DevBuf<int32_t>> grid;    // per level: Morton key -> box, or -1
};

void build_tree(const double* pts_user, int64_t n, const double lo[3],
                const double hi[3], int levels, hipStream_t s, int64_t* tally,
                DevTree& T);

// ------------------------------------------------------ geometry constants
// Per-plan constants of the interpolation (reference Chebyshev nodes on
// [-1,1], Lagrange weights, 1D child transfer matrices).
constexpr int kMaxM1 = 9;  // m + 1 <= 9
struct Interp {
  int m1 = 0;               // m + 1
  int K = 0;                // (m+1)^3
  int Kp = 0;               // K padded for the coupling kernels
  double node[kMaxM1];      // x_nu = cos((2 nu - 1) pi / (2(m+1)))
  double wgt[kMaxM1];       // 1 / prod_{mu != nu} (x_nu - x_mu)
  double E1[2][kMaxM1][kMaxM1];  // E1[b][j][k] = l_k((x_j + 2b - 1) / 2)
};

}  // namespace fdm
