// Internal definitions shared by the host planner and the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>

#include "../../include/tn.h"

namespace tn {

constexpr int kMaxAxes = TN_MAX_RANK;

// One index group (the M, N or K index of a contraction, or the output /
// summed index of a reduction) as a list of axes, innermost last.  Index
// value i decomposes into per-axis digits; each of up to three tensors
// addresses the group with its own stride per axis.  Division by an axis
// dimension uses a precomputed multiply-high (Granlund and Montgomery,
// PLDI 1994): q = (umulhi(n, mul) + n) >> shr, exact for n < 2^31.
struct Group {
  int32_t n;
  uint32_t dim[kMaxAxes];
  uint32_t mul[kMaxAxes];
  uint32_t shr[kMaxAxes];
  int64_t s[3][kMaxAxes];
};

__host__ __device__ inline uint32_t fast_div(uint32_t n, uint32_t mul, uint32_t shr) {
#if defined(__HIP_DEVICE_COMPILE__)
  return (__umulhi(n, mul) + n) >> shr;
#else
  return (uint32_t)((((uint64_t)n * mul) >> 32) + n) >> shr;
#endif
}

// Offsets of index `idx` in tensors 0..2 of the group (only the first `nt` are formed).
template <int NT>
__host__ __device__ inline void group_offsets(const Group& g, uint32_t idx, int64_t (&o)[NT], int first = 0) {
#pragma unroll
  for (int t = 0; t < NT; ++t) o[t] = 0;
#pragma unroll
  for (int i = kMaxAxes - 1; i >= 0; --i) {
    if (i < g.n) {
      uint32_t q = fast_div(idx, g.mul[i], g.shr[i]);
      uint32_t r = idx - q * g.dim[i];
#pragma unroll
      for (int t = 0; t < NT; ++t) o[t] += (int64_t)r * g.s[first + t][i];
      idx = q;
    }
  }
}

// Contraction GEMM descriptor: C[m, n] = sum_k A[m, k] B[k, n] over strided views.
//   gm: strides (A, C, -)   gn: strides (B, C, -)   gk: strides (A, B, -)
// LOAD_MNSCALAR: innermost row index unit-stride but not 16-byte loadable:
// scalar loads with the lanes of a wavefront along the rows
enum LoadMode : int32_t { LOAD_GENERIC = 0, LOAD_KVEC = 1, LOAD_MNVEC = 2, LOAD_MNSCALAR = 3 };
enum StoreMode : int32_t { STORE_SCALAR = 0, STORE_MVEC = 1 };

struct GemmDesc {
  const float* a;
  const float* b;
  float* c;
  int32_t M, N, K;
  int32_t a_mode, b_mode, c_mode;
  int32_t batch;
  int64_t a_bs, b_bs, c_bs;       // batch strides (elements)
  const uint32_t* a_scale_bits;   // nullable, per batch: A is multiplied by 2^-e(max) (exact)
  uint32_t* c_absmax;             // nullable, per batch: atomic max of |C| bit patterns
  int32_t tiles_m, tiles_n;
  Group gm, gn, gk;
};

// Strided reduction / elementwise descriptor:
//   out[r] = sum_k X[x(r) + x(k)] * (Y ? Y[y(r) + y(k)] : 1)
//   gr: strides (X, Y, out)   gk: strides (X, Y, -)
struct ReduceDesc {
  const float* x;
  const float* y;
  float* out;
  int64_t R, K;
  int32_t mode;        // 0: thread per output, 1: wave per output, 2: block per output, 3: four outputs per thread
  int32_t bf16_round;  // round operands to BF16 before the product
  int32_t kcontig;     // k is one unit-stride axis of X (and of Y)
  Group gr, gk;
};

// Host helpers (plan.cpp)
void set_fast_div(Group& g);

struct Err {
  int32_t code;
};

void set_error(const char* fmt, ...);
int32_t fail(int32_t code, const char* fmt, ...);
int32_t hip_check(hipError_t e, const char* what);

}  // namespace tn

#define TN_TRY(expr)               \
  do {                             \
    int32_t _s = (expr);           \
    if (_s != TN_OK) return _s;    \
  } while (0)
