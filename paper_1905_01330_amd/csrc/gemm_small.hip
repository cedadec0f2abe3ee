// Contractions whose contracted and one free extent are both tiny (an MPO
// acting on a bond pair, a 2-index gate): C[m, n] = sum_k A[m, k] B[k, n]
// with K <= 32 and N <= 16.  No matrix-core tile fits such a shape; the
// work is reading A and writing C once, so it is bound by HBM.  B lives in
// LDS, each thread owns one row m (consecutive m are the unit-stride index
// when there is one) and keeps its N sums in FP64.
#include "internal.h"

namespace tn {

constexpr int kSmallK = 32, kSmallN = 16;

__device__ inline float small_bf16(float x) { return (float)(__bf16)x; }

// PRELOAD: a row's K values are loaded before the first is used (for grids
// too small to hide one load at a time behind other waves; a full chip
// hides it, and there the extra registers would cost waves)
template <bool PRELOAD>
__global__ void __launch_bounds__(256) gemm_small_kernel(const GemmDesc d, int bf16_round) {
  __shared__ float sb[kSmallK * kSmallN];
  __shared__ int64_t ka[kSmallK];
  __shared__ int64_t cn[kSmallN];
  const int K = d.K, N = d.N;
  for (int e = threadIdx.x; e < K * N; e += blockDim.x) {
    const int k = e / N, n = e % N;
    int64_t ok[2], on[2];
    group_offsets<2>(d.gk, (uint32_t)k, ok, 0);
    group_offsets<2>(d.gn, (uint32_t)n, on, 0);
    float v = d.b[ok[1] + on[0]];
    sb[e] = bf16_round ? small_bf16(v) : v;
  }
  for (int k = threadIdx.x; k < K; k += blockDim.x) {
    int64_t ok[2];
    group_offsets<2>(d.gk, (uint32_t)k, ok, 0);
    ka[k] = ok[0];
  }
  for (int n = threadIdx.x; n < N; n += blockDim.x) {
    int64_t on[2];
    group_offsets<2>(d.gn, (uint32_t)n, on, 0);
    cn[n] = on[1];
  }
  __syncthreads();
  const int64_t nthreads = (int64_t)gridDim.x * blockDim.x;
  for (int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; m < d.M; m += nthreads) {
    int64_t om[2];
    group_offsets<2>(d.gm, (uint32_t)m, om, 0);
    double acc[kSmallN];
#pragma unroll
    for (int n = 0; n < kSmallN; ++n) acc[n] = 0.0;
    if constexpr (PRELOAD) {
      float av[kSmallK];
#pragma unroll
      for (int k = 0; k < kSmallK; ++k) av[k] = k < K ? d.a[om[0] + ka[k]] : 0.0f;
#pragma unroll
      for (int k = 0; k < kSmallK; ++k) {
        if (k < K) {
          const float a = bf16_round ? small_bf16(av[k]) : av[k];
#pragma unroll
          for (int n = 0; n < kSmallN; ++n)
            if (n < N) acc[n] += (double)a * (double)sb[k * N + n];
        }
      }
    } else {
      for (int k = 0; k < K; ++k) {
        float a = d.a[om[0] + ka[k]];
        if (bf16_round) a = small_bf16(a);
#pragma unroll
        for (int n = 0; n < kSmallN; ++n)
          if (n < N) acc[n] += (double)a * (double)sb[k * N + n];
      }
    }
#pragma unroll
    for (int n = 0; n < kSmallN; ++n)
      if (n < N) d.c[om[1] + cn[n]] = (float)acc[n];
  }
}

bool gemm_small_fits(const GemmDesc& d) {
  const bool n_small = d.K <= kSmallK && d.N <= kSmallN;
  const bool m_small = d.K <= kSmallK && d.M <= kSmallN;
  return d.batch == 1 && !d.a_scale_bits && !d.c_absmax && (n_small || m_small) && (int64_t)d.M * d.N >= 4096;
}

int32_t launch_gemm_small(const GemmDesc& d0, int32_t prec, hipStream_t st) {
  GemmDesc d = d0;
  if (!(d.K <= kSmallK && d.N <= kSmallN)) {
    // C^T = B^T A^T: the small free extent becomes N
    std::swap(d.a, d.b);
    std::swap(d.M, d.N);
    std::swap(d.gm, d.gn);
    for (int i = 0; i < d.gk.n; ++i) std::swap(d.gk.s[0][i], d.gk.s[1][i]);
  }
  int64_t blocks = (d.M + 255) / 256;
  blocks = blocks < 1 ? 1 : (blocks > 65536 ? 65536 : blocks);
  const int bf = prec == TN_PREC_BF16 ? 1 : 0;
  if (blocks < 256)
    hipLaunchKernelGGL(gemm_small_kernel<true>, dim3((unsigned)blocks), dim3(256), 0, st, d, bf);
  else
    hipLaunchKernelGGL(gemm_small_kernel<false>, dim3((unsigned)blocks), dim3(256), 0, st, d, bf);
  return hip_check(hipGetLastError(), "small gemm launch");
}

}  // namespace tn
