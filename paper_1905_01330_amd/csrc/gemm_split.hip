// Instantiation table of the lean-stage split-BF16 contraction kernels.
#include "gemm_inst_decl.h"
#include "gemm_split_kernel.h"

namespace tn {

// kind 1: both operands split into LDS, 160 x 256 tile, eight waves;
// kind 2: B private to each wave, 160 x 256, eight waves;
// kind 3: B private, 160 x 128 tile in two k groups of four waves.
GemmFn split_fn(int kind, int bmode) {
  const bool mn = bmode == LOAD_MNVEC;
  switch (kind) {
    case 1: return mn ? split_gemm_kernel<160, 256, 8, LOAD_MNVEC> : split_gemm_kernel<160, 256, 8, LOAD_KVEC>;
    case 2: return mn ? split_gemm_p_kernel<160, 256, LOAD_MNVEC, 1> : split_gemm_p_kernel<160, 256, LOAD_KVEC, 1>;
    default: return mn ? split_gemm_p_kernel<160, 128, LOAD_MNVEC, 2> : split_gemm_p_kernel<160, 128, LOAD_KVEC, 2>;
  }
}

}  // namespace tn

namespace tn {

// Matrix-core rate of the split-BF16 product pattern with register operands:
// 256 workgroups of eight waves; each wave runs five 32 x 32 blocks over
// n_steps k-steps of 16, the six term products of a block per step in a
// zero-based chain added to the block's accumulator every two steps, as the
// contraction kernels do, but with no loads and no LDS traffic.  The operand
// bits come from a hash of the lane and block (random mantissas, exponents
// near 1) or are all zero.  What it measures is how fast the chip runs this
// pattern of matrix-core work, which bounds the contraction kernels.
__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(2, 2)))
    split_mfma_rate_kernel(float* out, int n_steps, int zero) {
  constexpr int TM = 5;
  const int tid = threadIdx.x + blockIdx.x * 512;
  bf16x8_t a[TM][3], b[3];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int p = 0; p < 3; ++p) {
      u32x4_t u;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        uint32_t h = (uint32_t)tid * 2654435761u ^ (uint32_t)((i * 3 + p) * 40503 + q * 977);
        h ^= h >> 13;
        h *= 0x5bd1e995u;
        h ^= h >> 15;
        u[q] = zero ? 0u : ((h & 0x3fff3fffu) | 0x3c003c00u);
      }
      a[i][p] = __builtin_bit_cast(bf16x8_t, u);
    }
#pragma unroll
  for (int p = 0; p < 3; ++p) b[p] = a[p][2 - p];
  float one;
  asm("v_mov_b32 %0, 1.0" : "=v"(one));
  const f32x16_t z = {};
  f32x16_t acc[TM];
#pragma unroll
  for (int i = 0; i < TM; ++i) acc[i] = z;
  for (int s = 0; s < n_steps; s += 2) {
#pragma unroll
    for (int i = 0; i < TM; ++i) {
      f32x16_t t;
#pragma unroll
      for (int kc = 0; kc < 2; ++kc)
#pragma unroll
        for (int q = 0; q < 6; ++q) {
          const int pa = q == 0 ? 1 : q == 1 ? 0 : q == 2 ? 2 : q == 3 ? 0 : q == 4 ? 1 : 0;
          const int pb = q == 0 ? 1 : q == 1 ? 2 : q == 2 ? 0 : q == 3 ? 1 : q == 4 ? 0 : 0;
          t = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[i][pa], b[pb], (kc == 0 && q == 0) ? z : t, 0, 0, 0);
        }
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[i][r] = __builtin_fmaf(t[r], one, acc[i][r]);
    }
  }
  float sum = 0.f;
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int r = 0; r < 16; ++r) sum += acc[i][r];
  out[tid] = sum;
}

}  // namespace tn

extern "C" int32_t tn_measure_split_mfma_rate(int32_t n_steps, int32_t zero_operands, float* out, void* stream) {
  if (!out) return tn::fail(TN_ERR_INVALID_ARGUMENT, "out is NULL");
  if (n_steps < 2 || n_steps % 2 != 0) return tn::fail(TN_ERR_INVALID_ARGUMENT, "n_steps must be even and >= 2");
  hipLaunchKernelGGL(tn::split_mfma_rate_kernel, dim3(256), dim3(512), 0, static_cast<hipStream_t>(stream), out, n_steps,
                     zero_operands ? 1 : 0);
  return tn::hip_check(hipGetLastError(), "split_mfma_rate launch");
}
