// Low-rank coupling step (Sect. 2.7 with Alg. 4's M2L): each stored coupling
// matrix is held as its adaptive cross approximation A~ ~ U Vt (aca.hip), and
// a block's product A~ v~ is taken in two stages on the matrix cores,
//   T = Vt v~   (r x 1 per block),   g~ += U T,
// which costs 16 K r instead of 8 K^2 flops per block at rank r.
//
// Work units: an item's offsets are ordered by rank (highest first) and cut
// into groups of 16; one launch pair covers one group of many items, so that
// every group's T fits the plan's buffer and no two workgroups of a launch
// add into the same result.  A group runs at its padded rank rp (its first
// offset's rank rounded up to 16; stored in the item's `first` field as
// rp / 16 above the first-part bit): T rows and U columns beyond the rank
// are zero, so the padding changes no value.  `compact` holds the group's
// place in T, in units of 64 columns x 16 ranks.
//
// Stage 1 items (this file): a workgroup of 2 waves owns the 64 target
// slots of a group; for each of its offsets it gathers the source moment
// columns (as the dense items do), multiplies them by Vt of that offset
// (wave w: slot tile w, 1 or 2 rank tiles of 32; FP32 MFMA with FP32 sums)
// and writes the rp x 64 result to T, every slot's column (zero where the
// source box is empty).  Stage 2 items are the FP32 item of m2l_device.hpp
// with the U factor as its matrix and T as its columns, read by address
// (FP32 per-offset sums, FP32 totals of the group, FP64 result).
#include "m2l_device.hpp"

namespace fdm {

namespace {

constexpr int kAca1Threads = 128;  // 2 waves: one per 32-slot tile

// Moment slab of 64 columns x 16 k, staged by 128 threads (4 pieces each).
struct Slab64 {
  float4 v[4];
};

__device__ __forceinline__ Slab64 load_slab64(const TargetTile<64>& S, int colbuf,
                                              const float* __restrict__ mom, int k0) {
  Slab64 r;
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int e = threadIdx.x + kAca1Threads * u;  // piece: column e / 8, k 2 (e % 8) ..
    const int64_t col = S.col[colbuf][e / 8];
    r.v[u] = col >= 0 ? gload16<float4>(mom + 2 * (col + k0) + (e % 8) * 4) : float4{};
  }
  return r;
}

__device__ __forceinline__ void store_slab64(F32Shared<64>& sh, int buf, const Slab64& r) {
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int e = threadIdx.x + kAca1Threads * u;
    const int j = e / 8, k = 2 * (e % 8);
    sh.B[buf][0][k][j] = r.v[u].x;
    sh.B[buf][1][k][j] = r.v[u].y;
    sh.B[buf][0][k + 1][j] = r.v[u].z;
    sh.B[buf][1][k + 1][j] = r.v[u].w;
  }
}

// Vt operands of one slab for rank tile rt: lane (rank r, half kl) holds
// k = k0 + 8 kl + t at MFMA step t; Vt(r, k) at k * kp + r.
__device__ __forceinline__ void load_vt(float (&a)[2][8], const float* __restrict__ Vt,
                                        int64_t per, int k0, int kp, int rt, int lane) {
  const int r = 32 * rt + lane % 32, kl = lane / 32;
#pragma unroll
  for (int t = 0; t < 8; ++t) {
    const int ka = (k0 + 8 * kl + t) * kp + r;
    a[0][t] = gmem(Vt)[ka];
    a[1][t] = gmem(Vt)[per + ka];
  }
}

__device__ __forceinline__ void mfma_vt(f16v& acr, f16v& aci, const float (&a)[2][8],
                                        const F32Shared<64>& sh, int buf, int cl, int kl) {
#pragma unroll
  for (int t = 0; t < 8; ++t) {
    const float b_r = sh.B[buf][0][t + 8 * kl][cl];
    const float b_i = sh.B[buf][1][t + 8 * kl][cl];
    acr = __builtin_amdgcn_mfma_f32_32x32x2f32(a[0][t], b_r, acr, 0, 0, 0);
    acr = __builtin_amdgcn_mfma_f32_32x32x2f32(-a[1][t], b_i, acr, 0, 0, 0);
    aci = __builtin_amdgcn_mfma_f32_32x32x2f32(a[0][t], b_i, aci, 0, 0, 0);
    aci = __builtin_amdgcn_mfma_f32_32x32x2f32(a[1][t], b_r, aci, 0, 0, 0);
  }
}

// A wave's rows of one rank tile of T for its column: rows below rp.
__device__ __forceinline__ void store_t(float2* col, const f16v& acr, const f16v& aci, int rt,
                                        int rp, int lane) {
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    const int r = 32 * rt + 8 * (i / 4) + 4 * (lane / 32) + (i % 4);
    if (r < rp) col[r] = make_float2(acr[i], aci[i]);
  }
}

// Stage 1 of one group: for each offset v, T[v] = Vt_v M_v (rp x 64).
__device__ __forceinline__ void item_aca1(F32Shared<64>& sh, const M2LItem& it,
                                          const M2LDesc& D, int Kp) {
  using Tr = F32Traits;
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  load_targets(sh.S, it, D);
  __syncthreads();
  const int nv = it.vo_count;
  if (nv == 0) return;
  const int kp = D.kp;
  const int rp = 16 * (it.first >> 1);  // padded rank of the group: 16, 32, 48 or 64
  const bool two = rp > 32;              // a second rank tile
  const float* mom = static_cast<const float*>(D.mom);
  const float* bank = static_cast<const float*>(D.bank);
  float2* T = static_cast<float2*>(D.out) + int64_t(it.compact) * 1024;
  const int64_t per = int64_t(Kp) * kp;  // one plane of U or Vt
  const int ns = Kp / Tr::KS;
  const int total = nv * ns;
  const int kl = lane / 32, cl = 32 * wave + lane % 32;
  int4 od_cur = offset_of(D, it.vo_begin);
  int4 od_next = od_cur;
  source_columns(sh.S, 0, D, od_cur, it.c, Kp);
  __syncthreads();
  store_slab64(sh, 0, load_slab64(sh.S, 0, mom, 0));
  __syncthreads();
  f16v acr0, aci0, acr1, aci1;
  for (int q = 0; q < total; ++q) {
    const int v = q / ns, s = q % ns, cur = q & 1;
    if (s == 0) {
      od_cur = od_next;
      if (v + 1 < nv) {
        od_next = offset_of(D, it.vo_begin + v + 1);
        source_columns(sh.S, (v + 1) & 1, D, od_next, it.c, Kp);
      }
      acr0 = f16v{};
      aci0 = f16v{};
      acr1 = f16v{};
      aci1 = f16v{};
    }
    const bool more = q + 1 < total;
    Slab64 nxt{};
    if (more) nxt = load_slab64(sh.S, ((q + 1) / ns) & 1, mom, ((q + 1) % ns) * Tr::KS);
    // Vt planes follow the two U planes of the matrix's bank entry
    const float* Vt = bank + (od_cur.w >> 1) * 4 * per + 2 * per;
    float a0[2][8], a1[2][8];
    load_vt(a0, Vt, per, s * Tr::KS, kp, 0, lane);
    if (two) load_vt(a1, Vt, per, s * Tr::KS, kp, 1, lane);
    __builtin_amdgcn_sched_barrier(0);
    mfma_vt(acr0, aci0, a0, sh, cur, cl, kl);
    if (two) mfma_vt(acr1, aci1, a1, sh, cur, cl, kl);
    if (s == ns - 1) {  // the offset's T columns: rp ranks each
      float2* col = T + (int64_t(v) * 64 + cl) * rp;
      store_t(col, acr0, aci0, 0, rp, lane);
      if (two) store_t(col, acr1, aci1, 1, rp, lane);
    }
    if (more) store_slab64(sh, cur ^ 1, nxt);
    __syncthreads();
  }
}

template <bool QUEUE>
__global__ void __launch_bounds__(kAca1Threads) __attribute__((amdgpu_waves_per_eu(3)))
    k_m2l_aca1(const M2LItem* __restrict__ items, int64_t n_items,
               const M2LDesc* __restrict__ descs, int32_t* head, int Kp) {
  __shared__ F32Shared<64> sh;
  __shared__ int32_t next;
  run_items<QUEUE, false>(items, n_items, descs, nullptr, head, next,
                          [&](const M2LItem& it, const M2LDesc& D) { item_aca1(sh, it, D, Kp); });
}

template <bool QUEUE, int MAXT>
__global__ void __launch_bounds__(MAXT)
    k_m2l_aca2(const M2LItem* __restrict__ items, int64_t n_items,
               const M2LDesc* __restrict__ descs, int32_t* head, int Kp) {
  __shared__ F32Shared<64> sh;
  __shared__ int32_t next;
  run_items<QUEUE, false>(items, n_items, descs, nullptr, head, next,
                          [&](const M2LItem& it, const M2LDesc& D) {
                            item_f32<64, false, true>(sh, it, D, Kp);
                          });
}

template <class KG, class KQ>
void launch_aca_pair(KG grid_kernel, KQ queue_kernel, const M2LLaunch& L, int threads, int Kp,
                     bool persistent, int32_t* head, hipStream_t s, const char* name) {
  const int64_t n = L.n_items;
  if (persistent) {
    if (L.resident_wgs <= 0) fail(FDM_ERR_STATE, "persistent launch without a grid size");
    const unsigned grid = static_cast<unsigned>(std::min<int64_t>(n, L.resident_wgs));
    queue_kernel<<<grid, threads, 0, s>>>(L.items.get(), n, L.descs.get(), head, Kp);
  } else {
    grid_kernel<<<static_cast<unsigned>(n), threads, 0, s>>>(L.items.get(), n, L.descs.get(),
                                                             nullptr, Kp);
  }
  FDM_LAUNCH(name);
}

}  // namespace

void launch_items_aca(const M2LLaunch& L, int stage, int Kp, bool persistent, int32_t* head,
                      hipStream_t s) {
  if (stage == 1) {
    launch_aca_pair(k_m2l_aca1<false>, k_m2l_aca1<true>, L, kAca1Threads, Kp, persistent,
                    head, s, "k_m2l_aca1");
  } else if (m2l_threads(Kp) > 512) {
    launch_aca_pair(k_m2l_aca2<false, 768>, k_m2l_aca2<true, 768>, L, m2l_threads(Kp), Kp,
                    persistent, head, s, "k_m2l_aca2");
  } else {
    launch_aca_pair(k_m2l_aca2<false, 512>, k_m2l_aca2<true, 512>, L, m2l_threads(Kp), Kp,
                    persistent, head, s, "k_m2l_aca2");
  }
}

int64_t resident_aca(int stage, int Kp) {
  if (stage == 1) return resident_groups(k_m2l_aca1<true>, kAca1Threads);
  if (m2l_threads(Kp) > 512) return resident_groups(k_m2l_aca2<true, 768>, m2l_threads(Kp));
  return resident_groups(k_m2l_aca2<true, 512>, m2l_threads(Kp));
}

}  // namespace fdm
