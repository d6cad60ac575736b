// Low-rank coupling step (Sect. 2.7 with Alg. 4's M2L): each stored coupling
// matrix is held as its adaptive cross approximation A~ ~ U Vt (aca.hip), and
// a block's product A~ v~ is taken in two stages on the matrix cores,
//   T = Vt v~   (kp x 1 per block),   g~ += U T,
// which costs 16 K kp instead of 8 K^2 flops per block.
//
// Stage 1 items (this file): a workgroup of 4 waves owns the 64 target slots
// of a coupling item; for each of the item's offsets it gathers the source
// moment columns (as the dense items do), multiplies them by Vt of that
// offset (2 row tiles of 32 ranks x 2 column tiles of 32 slots, one per
// wave, FP32 MFMA with FP32 sums) and writes the kp x 64 result to T at the
// item's offset entry.  Stage 2 items are the FP32 item of m2l_device.hpp
// with the U factor as its matrix and T as its columns (FP32 per-offset sums,
// FP32 totals of 16 offsets, FP64 result).  The coupling step runs both
// stages chunk by chunk over the plan's items, T holding one chunk.
#include "m2l_device.hpp"

namespace fdm {

namespace {

constexpr int kAca1Threads = 256;  // 4 waves: (rank tile, slot tile)

// Moment slab of 64 columns x 16 k, staged by 256 threads (2 pieces each).
struct Slab64 {
  float4 v[2];
};

__device__ __forceinline__ Slab64 load_slab64(const TargetTile<64>& S, int colbuf,
                                              const float* __restrict__ mom, int k0) {
  Slab64 r;
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    const int e = threadIdx.x + kAca1Threads * u;  // piece: column e / 8, k 2 (e % 8) ..
    const int64_t col = S.col[colbuf][e / 8];
    r.v[u] = col >= 0 ? gload16<float4>(mom + 2 * (col + k0) + (e % 8) * 4) : float4{};
  }
  return r;
}

__device__ __forceinline__ void store_slab64(F32Shared<64>& sh, int buf, const Slab64& r) {
#pragma unroll
  for (int u = 0; u < 2; ++u) {
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

// Stage 1 of one item: for each offset v, T[pair v] = Vt_v M_v (kp x 64).
__device__ __forceinline__ void item_aca1(F32Shared<64>& sh, const M2LItem& it,
                                          const M2LDesc& D, int Kp) {
  using Tr = F32Traits;
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  const int rt = wave / 2, ct = wave % 2;  // rank tile, slot tile of this wave
  load_targets(sh.S, it, D);
  __syncthreads();
  const int nv = it.vo_count;
  if (nv == 0) return;
  const int kp = D.kp;
  const float* mom = static_cast<const float*>(D.mom);
  const float* bank = static_cast<const float*>(D.bank);
  float2* T = static_cast<float2*>(D.out);
  const int64_t per = int64_t(Kp) * kp;  // one plane of U or Vt
  const int ns = Kp / Tr::KS;
  const int total = nv * ns;
  int4 od_cur = offset_of(D, it.vo_begin);
  int4 od_next = od_cur;
  source_columns(sh.S, 0, D, od_cur, it.c, Kp);
  __syncthreads();
  store_slab64(sh, 0, load_slab64(sh.S, 0, mom, 0));
  __syncthreads();
  f16v acr, aci;
  for (int q = 0; q < total; ++q) {
    const int v = q / ns, s = q % ns, cur = q & 1;
    if (s == 0) {
      od_cur = od_next;
      if (v + 1 < nv) {
        od_next = offset_of(D, it.vo_begin + v + 1);
        source_columns(sh.S, (v + 1) & 1, D, od_next, it.c, Kp);
      }
      acr = f16v{};
      aci = f16v{};
    }
    const bool more = q + 1 < total;
    Slab64 nxt{};
    if (more) nxt = load_slab64(sh.S, ((q + 1) / ns) & 1, mom, ((q + 1) % ns) * Tr::KS);
    if (32 * rt < kp) {
      float a[2][8];
      // Vt planes follow the two U planes of the matrix's bank entry
      load_vt(a, bank + (od_cur.w >> 1) * 4 * per + 2 * per, per, s * Tr::KS, kp, rt, lane);
      __builtin_amdgcn_sched_barrier(0);
      const int kl = lane / 32, cl = 32 * ct + lane % 32;
#pragma unroll
      for (int t = 0; t < 8; ++t) {
        const float b_r = sh.B[cur][0][t + 8 * kl][cl];
        const float b_i = sh.B[cur][1][t + 8 * kl][cl];
        acr = __builtin_amdgcn_mfma_f32_32x32x2f32(a[0][t], b_r, acr, 0, 0, 0);
        acr = __builtin_amdgcn_mfma_f32_32x32x2f32(-a[1][t], b_i, acr, 0, 0, 0);
        aci = __builtin_amdgcn_mfma_f32_32x32x2f32(a[0][t], b_i, aci, 0, 0, 0);
        aci = __builtin_amdgcn_mfma_f32_32x32x2f32(a[1][t], b_r, aci, 0, 0, 0);
      }
      if (s == ns - 1) {  // the offset's T tile: column (pair, slot), kp ranks each
        float2* col = T + ((int64_t(it.vo_begin) + v) * 64 + cl) * kp;
#pragma unroll
        for (int i = 0; i < 16; ++i) {
          const int r = 32 * rt + 8 * (i / 4) + 4 * (lane / 32) + (i % 4);
          col[r] = make_float2(acr[i], aci[i]);
        }
      }
    }
    if (more) store_slab64(sh, cur ^ 1, nxt);
    __syncthreads();
  }
}

template <bool QUEUE>
__global__ void __launch_bounds__(kAca1Threads)
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
