// Kernel instantiation tables for the contraction GEMM (one translation unit
// per precision so the instantiations compile in parallel).
#pragma once

#include "gemm_inst_decl.h"
#include "gemm_kernel.h"

namespace tn {

// Waves per SIMD to hold the register budget to: what the LDS footprint
// allows (160 KB per CU, four SIMDs), capped at 2, and 1 when a wave's
// accumulators (plus the split precisions' temporaries) exceed 128 registers,
// where a smaller budget would only spill.
template <int P, int BM, int BN, int BK, int WM, int WN, int AMODE, int BMODE, int WK>
constexpr int lds_waves_per_simd() {
  using T = GemmTile<P, BM, BN, BK, WM, WN, AMODE, BMODE, WK>;
  constexpr int wg = (160 * 1024) / T::lds_bytes;
  constexpr int w = wg * WM * WN * WK / 4;
  constexpr int acc_regs = T::TM * T::TN * 16 + T::TMT * T::TNT * 16 * (PrecInfo<P>::planes > 1 ? 1 : 0) +
                           (T::CHAIN ? 32 : 0);
  if (acc_regs > 128) return 1;
  return w < 1 ? 1 : (w > 2 ? 2 : w);
}

template <int P, int BM, int BN, int BK, int WM, int WN, int AMODE, int BMODE, int WK = 1>
__global__ void __launch_bounds__(WM* WN * WK * 64)
    __attribute__((amdgpu_waves_per_eu(lds_waves_per_simd<P, BM, BN, BK, WM, WN, AMODE, BMODE, WK>())))
        gemm_kernel(const GemmDesc d) {
  __shared__ __attribute__((aligned(16))) char smem[GemmTile<P, BM, BN, BK, WM, WN, AMODE, BMODE, WK>::lds_bytes];
  __shared__ Group gk;
  if constexpr (AMODE < 0 || BMODE < 0) {
    copy_group(gk, d.gk);
    __syncthreads();
  }
  GemmTile<P, BM, BN, BK, WM, WN, AMODE, BMODE, WK>::run(d, gk, blockIdx.x, blockIdx.z, smem);
}

// Grouped launch: the workgroup finds its problem by binary search over the
// per-problem first-tile table, then expands the compact 2-D description
// into a full descriptor held in LDS.
// AMODE / BMODE as for gemm_kernel: the fast gathers when the host has
// checked that every problem of the launch has those layouts, else -1.
template <int P, int BM, int BN, int BK, int WM, int WN, int AMODE = -1, int BMODE = -1, int WK = 1>
__global__ void __launch_bounds__(WM* WN * WK * 64)
    gemm_grouped_kernel(const Gemm2D* probs, const int32_t* tile_start, int32_t n_probs) {
  __shared__ __attribute__((aligned(16))) char smem[GemmTile<P, BM, BN, BK, WM, WN, AMODE, BMODE, WK>::lds_bytes];
  __shared__ GemmDesc sd;
  __shared__ int32_t s_prob;
  const int bid = blockIdx.x;
  if (threadIdx.x == 0) {
    int lo = 0, hi = n_probs - 1;
    while (lo < hi) {
      int mid = (lo + hi + 1) >> 1;
      if (tile_start[mid] <= bid)
        lo = mid;
      else
        hi = mid - 1;
    }
    s_prob = lo;
    const Gemm2D& p = probs[lo];
    GemmDesc& d = sd;
    d.a = p.a;
    d.b = p.b;
    d.c = p.c;
    d.M = p.M;
    d.N = p.N;
    d.K = p.K;
    d.batch = 1;
    d.a_bs = d.b_bs = d.c_bs = 0;
    d.a_scale_bits = p.a_scale_bits;
    d.c_absmax = p.c_absmax;
    d.tiles_m = (p.M + BM - 1) / BM;
    d.tiles_n = (p.N + BN - 1) / BN;
    auto one = [](Group& g, int64_t dim, int64_t s0, int64_t s1) {
      g.n = 1;
      g.dim[0] = (uint32_t)dim;
      uint32_t shr = 0;
      while (shr < 32 && (1ull << shr) < (uint64_t)dim) ++shr;
      g.mul[0] = (uint32_t)((((1ull << 32) * ((1ull << shr) - (uint64_t)dim)) / (uint64_t)dim) + 1);
      g.shr[0] = shr;
      g.s[0][0] = s0;
      g.s[1][0] = s1;
      g.s[2][0] = 0;
    };
    one(d.gm, p.M, p.sam, p.scm);
    one(d.gn, p.N, p.sbn, p.scn);
    one(d.gk, p.K, p.sak, p.sbk);
    auto al = [](const void* q) { return (reinterpret_cast<uintptr_t>(q) & 15) == 0; };
    // the gather modes of the plan's rules (16-byte loads need 4-byte
    // alignment only; single axes take a partial last block)
    d.a_mode = p.sak == 1 ? LOAD_KVEC : p.sam == 1 ? LOAD_MNVEC : LOAD_GENERIC;
    d.b_mode = p.sbk == 1 ? LOAD_KVEC : p.sbn == 1 ? LOAD_MNVEC : LOAD_GENERIC;
    d.c_mode = (p.scm == 1 && p.M % 4 == 0 && p.scn % 4 == 0 && al(p.c)) ? STORE_MVEC : STORE_SCALAR;
  }
  __syncthreads();
  // a tile table built for another tile size must not reach past the problem
  const int tile = bid - tile_start[s_prob];
  if (tile >= sd.tiles_m * sd.tiles_n) return;
  GemmTile<P, BM, BN, BK, WM, WN, AMODE, BMODE, WK>::run(sd, sd.gk, tile, 0, smem);
}


template <int P, int AM, int BM_>
GemmFn gemm_fn_modes(int cfg) {
  switch (cfg) {
    case 0: return gemm_kernel<P, 256, 128, 16, 2, 2, AM, BM_>;
    case 1: return gemm_kernel<P, 128, 256, 16, 2, 2, AM, BM_>;
    case 2: return gemm_kernel<P, 128, 128, 16, 2, 2, AM, BM_>;
    case 3: return gemm_kernel<P, 128, 128, 32, 2, 2, AM, BM_>;
    case 4: return gemm_kernel<P, 128, 64, 32, 2, 2, AM, BM_>;
    case 5: return gemm_kernel<P, 64, 128, 32, 2, 2, AM, BM_>;
    case 6: return gemm_kernel<P, 64, 64, 32, 2, 2, AM, BM_>;
    case 8: return gemm_kernel<P, 160, 128, 16, 1, 4, AM, BM_>;
    case 9: return gemm_kernel<P, 128, 160, 16, 4, 1, AM, BM_>;
    case 10: return gemm_kernel<P, 160, 256, 32, 1, 8, AM, BM_>;
    case 11: return gemm_kernel<P, 256, 160, 32, 8, 1, AM, BM_>;
    case 12: return gemm_kernel<P, 128, 160, 32, 4, 1, AM, BM_, 2>;
    case 13: return gemm_kernel<P, 160, 128, 32, 1, 4, AM, BM_, 2>;
    case 14: return gemm_kernel<P, 64, 64, 64, 2, 2, AM, BM_, 2>;
    case 15: return gemm_kernel<P, 64, 64, 64, 2, 2, AM, BM_>;
    default: return gemm_kernel<P, 32, 32, 32, 1, 1, AM, BM_>;
  }
}

// variant 0: run-time gathers; 1..4: fast gathers (A, B) = (K,K) (K,MN) (MN,K) (MN,MN)
template <int P>
GemmFn gemm_fn(int cfg, int variant) {
  switch (variant) {
    case 1: return gemm_fn_modes<P, LOAD_KVEC, LOAD_KVEC>(cfg);
    case 2: return gemm_fn_modes<P, LOAD_KVEC, LOAD_MNVEC>(cfg);
    case 3: return gemm_fn_modes<P, LOAD_MNVEC, LOAD_KVEC>(cfg);
    case 4: return gemm_fn_modes<P, LOAD_MNVEC, LOAD_MNVEC>(cfg);
    default: return gemm_fn_modes<P, -1, -1>(cfg);
  }
}

template <int P, int AM, int BM_>
GroupedFn grouped_fn_modes(int cfg) {
  switch (cfg) {
    case 0: return gemm_grouped_kernel<P, 128, 128, 32, 2, 2, AM, BM_>;
    case 1: return gemm_grouped_kernel<P, 64, 64, 64, 2, 2, AM, BM_>;
    case 3: return gemm_grouped_kernel<P, 64, 64, 64, 2, 2, AM, BM_, 2>;
    // eight waves side by side: fast gathers only (the run-time gathers
    // exceed its register budget; such launches never take this tile)
    case 4:
      if constexpr (AM >= 0 && BM_ >= 0) return gemm_grouped_kernel<P, 160, 256, 32, 1, 8, AM, BM_>;
      else return gemm_grouped_kernel<P, 128, 128, 32, 2, 2, AM, BM_>;
    default: return gemm_grouped_kernel<P, 32, 32, 32, 1, 1, AM, BM_>;
  }
}

// variant as for gemm_fn: 0 run-time gathers; 1..4 (A, B) = (K,K) (K,MN) (MN,K) (MN,MN)
template <int P>
GroupedFn grouped_fn(int cfg, int variant) {
  switch (variant) {
    case 1: return grouped_fn_modes<P, LOAD_KVEC, LOAD_KVEC>(cfg);
    case 2: return grouped_fn_modes<P, LOAD_KVEC, LOAD_MNVEC>(cfg);
    case 3: return grouped_fn_modes<P, LOAD_MNVEC, LOAD_KVEC>(cfg);
    case 4: return grouped_fn_modes<P, LOAD_MNVEC, LOAD_MNVEC>(cfg);
    default: return grouped_fn_modes<P, -1, -1>(cfg);
  }
}

}  // namespace tn
