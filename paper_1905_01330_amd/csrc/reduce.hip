// Strided reductions and elementwise products: rank-0/1 contraction results
// (dot, matrix-vector), trace edges, outer products and permuting copies.
//   out[r] = sum_k X[x(r) + x(k)] * (Y ? Y[y(r) + y(k)] : 1)
// The sum is accumulated in FP64 (these kernels are bound by HBM bandwidth,
// so the wider accumulator costs nothing).  Three shapes of parallelism:
//   mode 0: one thread per output (many outputs or short sums);
//   mode 1: one 64-lane wavefront per output, lanes stride over k, then a
//           butterfly reduction across the wavefront;
//   mode 2: one 256-thread workgroup per output (few outputs, long sums),
//           wavefront reductions followed by an LDS reduction.
#include "internal.h"

namespace tn {

__device__ inline float bf16_rne(float x) { return (float)(__bf16)x; }

__device__ inline int64_t k_offset(const Group& g, int ti, uint32_t k) {
  if (g.n == 1) return (int64_t)k * g.s[ti][0];
  int64_t o[1];
  group_offsets<1>(g, k, o, ti);
  return o[0];
}

__device__ inline double partial_sum(const ReduceDesc& d, int64_t ox, int64_t oy, int64_t k0, int64_t kstep) {
  double acc = 0.0;
  for (int64_t k = k0; k < d.K; k += kstep) {
    float xv = d.x[ox + k_offset(d.gk, 0, (uint32_t)k)];
    float yv = d.y ? d.y[oy + k_offset(d.gk, 1, (uint32_t)k)] : 1.0f;
    if (d.bf16_round) {
      xv = bf16_rne(xv);
      yv = bf16_rne(yv);
    }
    acc += (double)xv * (double)yv;
  }
  return acc;
}

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__global__ void __launch_bounds__(256) reduce_kernel(const ReduceDesc d) {
  if (d.mode == 0) {
    const int64_t nthreads = (int64_t)gridDim.x * blockDim.x;
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < d.R; r += nthreads) {
      int64_t o[3];
      group_offsets<3>(d.gr, (uint32_t)r, o, 0);
      d.out[o[2]] = (float)partial_sum(d, o[0], o[1], 0, 1);
    }
  } else if (d.mode == 1) {
    const int lane = threadIdx.x & 63;
    const int64_t nwaves = (int64_t)gridDim.x * (blockDim.x >> 6);
    for (int64_t r = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6; r < d.R; r += nwaves) {
      int64_t o[3];
      group_offsets<3>(d.gr, (uint32_t)r, o, 0);
      double s = wave_sum(partial_sum(d, o[0], o[1], lane, 64));
      if (lane == 0) d.out[o[2]] = (float)s;
    }
  } else {
    __shared__ double part[4];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int64_t r = blockIdx.x; r < d.R; r += gridDim.x) {
      int64_t o[3];
      group_offsets<3>(d.gr, (uint32_t)r, o, 0);
      double s = wave_sum(partial_sum(d, o[0], o[1], threadIdx.x, blockDim.x));
      if (lane == 0) part[wave] = s;
      __syncthreads();
      if (threadIdx.x == 0) d.out[o[2]] = (float)(part[0] + part[1] + part[2] + part[3]);
      __syncthreads();
    }
  }
}

int32_t launch_reduce(ReduceDesc& d, hipStream_t st) {
  if (d.R >= (1ll << 31) || d.K >= (1ll << 31)) return fail(TN_ERR_UNSUPPORTED, "reduction larger than 2^31");
  if (d.R >= 4096 || d.K <= 16)
    d.mode = 0;
  else if (d.R >= 64)
    d.mode = 1;
  else
    d.mode = 2;
  int64_t blocks;
  if (d.mode == 0)
    blocks = (d.R + 255) / 256;
  else if (d.mode == 1)
    blocks = (d.R + 3) / 4;
  else
    blocks = d.R;
  if (blocks > 65536) blocks = 65536;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(reduce_kernel, dim3((unsigned)blocks), dim3(256), 0, st, d);
  return hip_check(hipGetLastError(), "reduce launch");
}

}  // namespace tn
