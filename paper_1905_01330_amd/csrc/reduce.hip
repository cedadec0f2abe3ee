// Strided reductions and elementwise products: rank-0/1 contraction results
// (dot, matrix-vector), trace edges, outer products and permuting copies.
//   out[r] = sum_k X[x(r) + x(k)] * (Y ? Y[y(r) + y(k)] : 1)
// The sum is accumulated in FP64 (these kernels are bound by HBM bandwidth,
// so the wider accumulator costs nothing).  Shapes of parallelism:
//   elementwise (K = 1): one thread per output, or four consecutive outputs
//     per thread (one 16-byte store) when the innermost output axis is
//     unit-stride in the output;
//   mode 0: one thread per output: when the outputs, not the summed index,
//     are unit-stride in X (column sums, traces over leading axes) or the
//     sums are short;
//   mode 3: as mode 0, four consecutive outputs per thread with 16-byte
//     loads, when the innermost output axis is unit-stride in X (and Y) and
//     its extent is a multiple of four;
//   mode 1: one 64-lane wavefront per output, lanes stride over k (16-byte
//     loads when k is one unit-stride axis of both operands), then a
//     butterfly reduction across the wavefront;
//   mode 2: one 256-thread workgroup per output (few outputs, no scratch);
//   split: few long unit-stride sums: the k range of each output is cut over
//     many workgroups, whose FP64 partials go to a small caller-provided
//     scratch; a second kernel adds each output's partials in a fixed order
//     (deterministic, no atomics).
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
#pragma unroll 4
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

typedef float f4_t __attribute__((ext_vector_type(4)));

// sum over k in [k0, k1) of x[k] * y[k] for unit-stride k, four k per lane
// step (16-byte loads when both rows are 16-byte aligned); lane-strided
__device__ inline double contig_sum(const ReduceDesc& d, const float* x, const float* y, int64_t k0, int64_t k1,
                                    int lane, int nlanes) {
  double acc = 0.0;
  const bool vec = ((reinterpret_cast<uintptr_t>(x + k0) & 15) == 0) &&
                   (!y || (reinterpret_cast<uintptr_t>(y + k0) & 15) == 0);
  int64_t k = k0;
  if (vec) {
    const int64_t n4 = (k1 - k0) / 4;
    auto quad = [&](int64_t i, double& a4) {
      f4_t xv = *reinterpret_cast<const f4_t*>(x + k0 + 4 * i);
      f4_t yv = y ? *reinterpret_cast<const f4_t*>(y + k0 + 4 * i) : f4_t{1.f, 1.f, 1.f, 1.f};
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        float a = xv[j], b = yv[j];
        if (d.bf16_round) {
          a = bf16_rne(a);
          b = bf16_rne(b);
        }
        a4 += (double)a * (double)b;
      }
    };
    // four independent partial sums (added in a fixed order at the end), so
    // four 16-byte loads per lane are in flight instead of one FP64 add chain
    double acc4[4] = {0.0, 0.0, 0.0, 0.0};
    int64_t i = lane;
    for (; i + 3 * nlanes < n4; i += 4 * nlanes) {
#pragma unroll
      for (int u = 0; u < 4; ++u) quad(i + u * nlanes, acc4[u]);
    }
    for (; i < n4; i += nlanes) quad(i, acc4[0]);
    acc = (acc4[0] + acc4[1]) + (acc4[2] + acc4[3]);
    k = k0 + 4 * n4;
  }
  for (int64_t i = k + lane; i < k1; i += nlanes) {
    float a = x[i], b = y ? y[i] : 1.0f;
    if (d.bf16_round) {
      a = bf16_rne(a);
      b = bf16_rne(b);
    }
    acc += (double)a * (double)b;
  }
  return acc;
}

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// sum over the workgroup (256 threads); the result is valid in thread 0
__device__ inline double block_sum(double v, double* part) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  v = wave_sum(v);
  if (lane == 0) part[wave] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0) s = part[0] + part[1] + part[2] + part[3];
  __syncthreads();
  return s;
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
      const double p = d.kcontig ? contig_sum(d, d.x + o[0], d.y ? d.y + o[1] : nullptr, 0, d.K, lane, 64)
                                 : partial_sum(d, o[0], o[1], lane, 64);
      const double s = wave_sum(p);
      if (lane == 0) d.out[o[2]] = (float)s;
    }
  } else {
    __shared__ double part[4];
    for (int64_t r = blockIdx.x; r < d.R; r += gridDim.x) {
      int64_t o[3];
      group_offsets<3>(d.gr, (uint32_t)r, o, 0);
      const double p = d.kcontig ? contig_sum(d, d.x + o[0], d.y ? d.y + o[1] : nullptr, 0, d.K, threadIdx.x, 256)
                                 : partial_sum(d, o[0], o[1], threadIdx.x, blockDim.x);
      const double s = block_sum(p, part);
      if (threadIdx.x == 0) d.out[o[2]] = (float)s;
    }
  }
}

// mode 3: four consecutive outputs per thread (its own kernel, so the wider
// registers do not lower the occupancy of the other modes).  KG > 1 splits
// each output's k range over KG threads of the workgroup (k = kg, kg + KG,
// ...) when the outputs alone give too few workgroups to keep the loads in
// flight; the KG partial sums are then added in the fixed order kg = 0, 1, ...
template <int KG>
__global__ void __launch_bounds__(256) reduce4_kernel(const ReduceDesc d) {
  constexpr int QPB = 256 / KG;   // quads of outputs per workgroup
  __shared__ double part[KG > 1 ? KG : 1][QPB][4];
  const int in = d.gr.n - 1;
  const int64_t so = d.gr.s[2][in];
  const int ql = threadIdx.x % QPB, kg = threadIdx.x / QPB;
  const int64_t nq = d.R / 4;
  for (int64_t base = (int64_t)blockIdx.x * QPB; base < nq; base += (int64_t)gridDim.x * QPB) {
    const int64_t q = base + ql;
    const bool valid = q < nq;
    int64_t o[3] = {0, 0, 0};
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    if (valid) {
      group_offsets<3>(d.gr, (uint32_t)(4 * q), o, 0);
#pragma unroll 4
      for (int64_t k = kg; k < d.K; k += KG) {
        const float* xp = d.x + o[0] + k_offset(d.gk, 0, (uint32_t)k);
        const float* yp = d.y ? d.y + o[1] + k_offset(d.gk, 1, (uint32_t)k) : nullptr;
        f4_t xv, yv = {1.f, 1.f, 1.f, 1.f};
        if ((reinterpret_cast<uintptr_t>(xp) & 15) == 0) {
          xv = *reinterpret_cast<const f4_t*>(xp);
        } else {
          xv = f4_t{xp[0], xp[1], xp[2], xp[3]};
        }
        if (yp) {
          if ((reinterpret_cast<uintptr_t>(yp) & 15) == 0)
            yv = *reinterpret_cast<const f4_t*>(yp);
          else
            yv = f4_t{yp[0], yp[1], yp[2], yp[3]};
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          float a = xv[j], b = yv[j];
          if (d.bf16_round) {
            a = bf16_rne(a);
            b = bf16_rne(b);
          }
          acc[j] += (double)a * (double)b;
        }
      }
    }
    if constexpr (KG > 1) {
#pragma unroll
      for (int j = 0; j < 4; ++j) part[kg][ql][j] = acc[j];
      __syncthreads();
      if (kg == 0) {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          double t = part[0][ql][j];
#pragma unroll
          for (int g = 1; g < KG; ++g) t += part[g][ql][j];
          acc[j] = t;
        }
      }
      __syncthreads();
    }
    if (valid && kg == 0) {
      if (so == 1 && (reinterpret_cast<uintptr_t>(d.out + o[2]) & 15) == 0) {
        *reinterpret_cast<f4_t*>(d.out + o[2]) = f4_t{(float)acc[0], (float)acc[1], (float)acc[2], (float)acc[3]};
      } else {
#pragma unroll
        for (int j = 0; j < 4; ++j) d.out[o[2] + j * so] = (float)acc[j];
      }
    }
  }
}

// split reduction, pass 1: workgroup (g, r) sums chunk g of output r's k range
__global__ void __launch_bounds__(256) reduce_partial_kernel(const ReduceDesc d, double* partial, int64_t chunk) {
  __shared__ double part[4];
  const int64_t r = blockIdx.y;
  const int g = blockIdx.x;
  int64_t o[3];
  group_offsets<3>(d.gr, (uint32_t)r, o, 0);
  const int64_t k0 = (int64_t)g * chunk;
  const int64_t k1 = k0 + chunk < d.K ? k0 + chunk : d.K;
  const double s = block_sum(contig_sum(d, d.x + o[0], d.y ? d.y + o[1] : nullptr, k0, k1, threadIdx.x, 256), part);
  if (threadIdx.x == 0) partial[r * gridDim.x + g] = s;
}

// split reduction, pass 2: one wavefront per output adds its G partials
__global__ void __launch_bounds__(64) reduce_final_kernel(const ReduceDesc d, const double* partial, int G) {
  const int64_t r = blockIdx.x;
  double s = 0.0;
  for (int g = threadIdx.x; g < G; g += 64) s += partial[r * G + g];
  s = wave_sum(s);
  if (threadIdx.x == 0) {
    int64_t o[3];
    group_offsets<3>(d.gr, (uint32_t)r, o, 0);
    d.out[o[2]] = (float)s;
  }
}

// elementwise products (K = 1), four consecutive outputs of the innermost
// output axis per thread: that axis is unit-stride in the output and its
// extent is a multiple of four, so the four never cross into the next row
__global__ void __launch_bounds__(256) elementwise4_kernel(const ReduceDesc d) {
  const int in = d.gr.n - 1;
  const int64_t sx = d.gr.s[0][in], sy = d.gr.s[1][in];
  const int64_t nq = d.R / 4;
  const int64_t nthreads = (int64_t)gridDim.x * blockDim.x;
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < nq; q += nthreads) {
    int64_t o[3];
    group_offsets<3>(d.gr, (uint32_t)(4 * q), o, 0);
    // the four inputs of each operand: one load when its stride is 0 (the
    // operand does not carry the innermost output axis), one 16-byte load
    // when it is 1 and aligned, else four
    auto four = [](const float* p, int64_t s) {
      if (s == 0) {
        const float t = *p;
        return f4_t{t, t, t, t};
      }
      if (s == 1 && (reinterpret_cast<uintptr_t>(p) & 15) == 0) return *reinterpret_cast<const f4_t*>(p);
      return f4_t{p[0], p[s], p[2 * s], p[3 * s]};
    };
    const f4_t xq = four(d.x + o[0], sx);
    const f4_t yq = d.y ? four(d.y + o[1], sy) : f4_t{1.f, 1.f, 1.f, 1.f};
    f4_t v;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      float xv = xq[j], yv = yq[j];
      if (d.bf16_round) {
        xv = bf16_rne(xv);
        yv = bf16_rne(yv);
      }
      v[j] = (float)((double)xv * (double)yv);
    }
    if ((reinterpret_cast<uintptr_t>(d.out + o[2]) & 15) == 0) {
      // streamed: the product is written once and not read back here
      __builtin_nontemporal_store(v, reinterpret_cast<f4_t*>(d.out + o[2]));
    } else {
#pragma unroll
      for (int j = 0; j < 4; ++j) d.out[o[2] + j] = v[j];
    }
  }
}

int32_t launch_reduce(ReduceDesc& d, void* scratch, size_t scratch_bytes, hipStream_t st) {
  if (d.R >= (1ll << 31) || d.K >= (1ll << 31)) return fail(TN_ERR_UNSUPPORTED, "reduction larger than 2^31");
  // k is one axis of unit stride in X (and in Y)
  d.kcontig = d.gk.n == 1 && d.gk.s[0][0] == 1 && (!d.y || d.gk.s[1][0] == 1) ? 1 : 0;
  const int in = d.gr.n - 1;
  if (d.K == 1) {
    const bool vec4 = d.gr.n >= 1 && d.gr.s[2][in] == 1 && d.gr.dim[in] % 4 == 0;
    int64_t blocks = ((vec4 ? d.R / 4 : d.R) + 255) / 256;
    blocks = blocks < 1 ? 1 : (blocks > 65536 ? 65536 : blocks);
    if (vec4) {
      hipLaunchKernelGGL(elementwise4_kernel, dim3((unsigned)blocks), dim3(256), 0, st, d);
    } else {
      d.mode = 0;
      hipLaunchKernelGGL(reduce_kernel, dim3((unsigned)blocks), dim3(256), 0, st, d);
    }
    return hip_check(hipGetLastError(), "elementwise launch");
  }
  // few long unit-stride sums: split over workgroups when scratch is given
  if (d.kcontig && d.R < 1024 && d.K >= 16384 && scratch) {
    int64_t G = (2048 + d.R - 1) / d.R;                 // about 2048 workgroups in all
    const int64_t gmax = (d.K + 4095) / 4096;           // at least 4096 k per workgroup
    if (G > gmax) G = gmax;
    if (G * d.R * 8 > (int64_t)scratch_bytes) G = (int64_t)scratch_bytes / (8 * d.R);
    if (G >= 2) {
      const int64_t chunk = ((d.K + G - 1) / G + 3) / 4 * 4;   // multiple of 4: 16-byte aligned chunk starts
      G = (d.K + chunk - 1) / chunk;
      double* partial = static_cast<double*>(scratch);
      hipLaunchKernelGGL(reduce_partial_kernel, dim3((unsigned)G, (unsigned)d.R), dim3(256), 0, st, d, partial, chunk);
      TN_TRY(hip_check(hipGetLastError(), "reduce launch"));
      hipLaunchKernelGGL(reduce_final_kernel, dim3((unsigned)d.R), dim3(64), 0, st, d, (const double*)partial, (int)G);
      return hip_check(hipGetLastError(), "reduce launch");
    }
  }
  // outputs unit-stride in X and k not: one thread per output keeps the loads coalesced
  const bool r_unit = d.gr.n >= 1 && d.gr.s[0][in] == 1 && !d.kcontig;
  const bool r_vec4 = r_unit && d.gr.dim[in] % 4 == 0 && (!d.y || d.gr.s[1][in] == 1);
  if (r_vec4)
    d.mode = 3;
  else if (d.K <= 16 || r_unit || (d.R >= 4096 && !d.kcontig))
    d.mode = 0;
  else if (d.R >= 64)
    d.mode = 1;
  else
    d.mode = 2;
  int64_t blocks;
  if (d.mode == 0)
    blocks = (d.R + 255) / 256;
  else if (d.mode == 3)
    blocks = (d.R / 4 + 255) / 256;
  else if (d.mode == 1)
    blocks = (d.R + 3) / 4;
  else
    blocks = d.R;
  // few workgroups of outputs and a k range worth splitting: four threads per output quad
  const bool ksplit = d.mode == 3 && blocks < 1024 && d.K >= 16;
  if (ksplit) blocks = (d.R / 4 + 63) / 64;
  if (blocks > 65536) blocks = 65536;
  if (blocks < 1) blocks = 1;
  if (d.mode == 3 && ksplit)
    hipLaunchKernelGGL(reduce4_kernel<4>, dim3((unsigned)blocks), dim3(256), 0, st, d);
  else if (d.mode == 3)
    hipLaunchKernelGGL(reduce4_kernel<1>, dim3((unsigned)blocks), dim3(256), 0, st, d);
  else
    hipLaunchKernelGGL(reduce_kernel, dim3((unsigned)blocks), dim3(256), 0, st, d);
  return hip_check(hipGetLastError(), "reduce launch");
}

}  // namespace tn
