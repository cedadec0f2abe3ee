// Chain networks of Fig. 3a: MPS inner products (single and uneven batches)
// and MPS-MPO-MPS environment sweeps.  Every site is a short sequence of
// contraction GEMMs; the inner product keeps its running environment in
// range with exact power-of-two rescaling fused into the GEMMs (the epilogue
// records max|E| with an atomic max, the next site's GEMM scales its result
// by 2^-e) and sums the exponents in FP64.  A single inner product of 4 or
// more sites runs its two halves from both ends on two streams.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <vector>

#include "internal.h"

namespace tn {

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// exponent e of a max-abs bit pattern such that the GEMM scaled by 2^-e (0 if unusable)
__device__ inline int scale_exponent(uint32_t bits) {
  int e = (int)((bits >> 23) & 0xffu);
  if (e == 0 || e > 253) return 0;
  return e - 127;
}

__global__ void mps_init_kernel(float* e0, uint32_t* slots, int n_slots) {
  for (int i = threadIdx.x + blockIdx.x * blockDim.x; i < n_slots; i += blockDim.x * gridDim.x)
    slots[i] = i == 0 ? 0x3f800000u : 0u;
  if (threadIdx.x == 0 && blockIdx.x == 0) e0[0] = 1.0f;
}

__global__ void mps_finish_kernel(const float* e_final, const uint32_t* slots, int n_used, double* out2) {
  __shared__ double part[4];
  double s = 0.0;
  for (int i = threadIdx.x; i < n_used; i += blockDim.x) s += (double)scale_exponent(slots[i]);
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) s += __shfl_xor(s, o, 64);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = part[0] + part[1] + part[2] + part[3];
    out2[0] = (double)e_final[0];
    out2[1] = t * 0.69314718055994530942;
  }
}

// Two-sided inner product: the left environment E_L at the middle bond and
// the right one E_R meet in <psi|phi> = sum_{a', a} E_L[a', a] E_R[a', a].
// Products of FP32 values are exact in FP64, so the FP64 sum needs neither
// environment's last scale; partial sums per workgroup, then a fixed-order
// total (deterministic).
__global__ void __launch_bounds__(256) env_dot_partial_kernel(const float* __restrict__ el,
                                                              const float* __restrict__ er, int64_t n, double* part) {
  __shared__ double red[4];
  double s = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
    s += (double)el[i] * (double)er[i];
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) s += __shfl_xor(s, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

// value = total * 2^(exponents applied on both sides), written as a mantissa
// in [0.5, 1) and a natural-log scale
__global__ void __launch_bounds__(256) env_dot_finish_kernel(const double* part, int n_part, const uint32_t* ls, int nl,
                                                             const uint32_t* rsl, int nr, double* out2) {
  __shared__ double red[2][4];
  double v = threadIdx.x < n_part ? part[threadIdx.x] : 0.0;
  double e = 0.0;
  for (int i = threadIdx.x; i < nl; i += 256) e += (double)scale_exponent(ls[i]);
  for (int i = threadIdx.x; i < nr; i += 256) e += (double)scale_exponent(rsl[i]);
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) {
    v += __shfl_xor(v, o, 64);
    e += __shfl_xor(e, o, 64);
  }
  if ((threadIdx.x & 63) == 0) {
    red[0][threadIdx.x >> 6] = v;
    red[1][threadIdx.x >> 6] = e;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const double total = red[0][0] + red[0][1] + red[0][2] + red[0][3];
    const double ex = red[1][0] + red[1][1] + red[1][2] + red[1][3];
    int e2 = 0;
    const double m = frexp(total, &e2);
    out2[0] = m;
    out2[1] = (ex + (double)e2) * 0.69314718055994530942;
  }
}

// ---------------------------------------------------------------------------
// validation helpers

static int32_t check_chain(int32_t n_sites, const tn_tensor* sites, const char* name, int32_t dtype,
                           std::vector<int64_t>* dims, int64_t* phys) {
  if (n_sites < 1) return fail(TN_ERR_INVALID_ARGUMENT, "n_sites must be >= 1");
  if (!sites) return fail(TN_ERR_INVALID_ARGUMENT, "%s is NULL", name);
  dims->clear();
  for (int k = 0; k < n_sites; ++k) {
    char nm[48];
    snprintf(nm, sizeof(nm), "%s[%d]", name, k);
    TN_TRY(check_tensor(&sites[k], nm, dtype));
    if (sites[k].rank != 3) return fail(TN_ERR_SHAPE_MISMATCH, "%s must be [D_k, d, D_k+1]", nm);
    if (k == 0) {
      if (sites[0].shape[0] != 1) return fail(TN_ERR_SHAPE_MISMATCH, "%s: first bond must be 1", name);
      *phys = sites[0].shape[1];
      dims->push_back(1);
    } else {
      if (sites[k].shape[0] != dims->back()) return fail(TN_ERR_SHAPE_MISMATCH, "%s: bond %d does not match", name, k);
    }
    if (sites[k].shape[1] != *phys) return fail(TN_ERR_SHAPE_MISMATCH, "%s: physical dimension differs", nm);
    dims->push_back(sites[k].shape[2]);
  }
  if (dims->back() != 1) return fail(TN_ERR_SHAPE_MISMATCH, "%s: last bond must be 1", name);
  return TN_OK;
}

// GEMM views of one inner-product site (shared by the single and batched paths)
//   T[a', s, b] = sum_a E[a', a] phi[a, s, b]        (E scaled by 2^-e of slot k)
//   E'[b', b]  = sum_{a', s} psi[a', s, b'] T[a', s, b]
static int32_t inner_site(const tn_tensor& psi, const tn_tensor& phi, float* e_in, float* e_out, float* t,
                          uint32_t* slots, int k, int32_t prec, hipStream_t st, float* sk = nullptr,
                          size_t sk_floats = 0) {
  SplitKScope slices(sk, sk_floats);
  const int64_t da = psi.shape[0], db = phi.shape[0], d = psi.shape[1];
  const int64_t da2 = psi.shape[2], db2 = phi.shape[2];
  tn_tensor e = make_view(e_in, TN_F32, {da, db});
  tn_tensor tv = make_view(t, TN_F32, {da, d, db2});
  tn_tensor eo = make_view(e_out, TN_F32, {da2, db2});
  const int32_t a1[1] = {1}, b1[1] = {0};
  GemmDesc g;
  TN_TRY(plan_gemm(e, phi, 1, a1, b1, tv, g));
  g.a_scale_bits = slots + k;
  TN_TRY(launch_gemm(g, prec, st));
  const int32_t a2[2] = {0, 1}, b2[2] = {0, 1};
  TN_TRY(plan_gemm(psi, tv, 2, a2, b2, eo, g));
  g.c_absmax = slots + k + 1;
  return launch_gemm(g, prec, st);
}

// right-to-left site of the two-sided inner product
//   T[a', s, b] = sum_b' psi[a', s, b'] E_R[b', b]   (scaled by 2^-e of in_slot:
//                                                      exact, so which factor carries it is immaterial)
//   E_R'[a', a] = sum_{s, b} T[a', s, b] phi[a, s, b]
static int32_t inner_site_right(const tn_tensor& psi, const tn_tensor& phi, float* e_in, float* e_out, float* t,
                                uint32_t* in_slot, uint32_t* out_slot, int32_t prec, hipStream_t st,
                                float* sk = nullptr, size_t sk_floats = 0) {
  SplitKScope slices(sk, sk_floats);
  const int64_t da = psi.shape[0], db = phi.shape[0], d = psi.shape[1];
  const int64_t da2 = psi.shape[2], db2 = phi.shape[2];
  tn_tensor e = make_view(e_in, TN_F32, {da2, db2});
  tn_tensor tv = make_view(t, TN_F32, {da, d, db2});
  tn_tensor eo = make_view(e_out, TN_F32, {da, db});
  const int32_t a1[1] = {2}, b1[1] = {0};
  GemmDesc g;
  TN_TRY(plan_gemm(psi, e, 1, a1, b1, tv, g));
  g.a_scale_bits = in_slot;
  TN_TRY(launch_gemm(g, prec, st));
  const int32_t a2[2] = {1, 2}, b2[2] = {1, 2};
  TN_TRY(plan_gemm(tv, phi, 2, a2, b2, eo, g));
  g.c_absmax = out_slot;
  return launch_gemm(g, prec, st);
}

// chains of at least this many sites are contracted from both ends at once
constexpr int kInnerTwoSided = 4;
constexpr int kEnvDotParts = 256;

struct InnerLayout {
  size_t e0, e1, t, slots, er0, er1, tr, rslots, part, sk, skr, total;
  size_t sk_floats;   // k-slice partials per end
};

static InnerLayout inner_layout(int32_t n, const std::vector<int64_t>& dp, const std::vector<int64_t>& dq, int64_t d) {
  int64_t me = 1, mt = 1;
  for (int k = 0; k <= n; ++k) me = std::max(me, dp[k] * dq[k]);
  for (int k = 0; k < n; ++k) mt = std::max(mt, dp[k] * d * dq[k + 1]);
  InnerLayout L;
  L.e0 = 0;
  L.e1 = align256(me * 4);
  L.t = L.e1 + align256(me * 4);
  L.slots = L.t + align256(mt * 4);
  L.er0 = L.slots + align256((size_t)(n + 1) * 4);
  L.er1 = L.er0 + align256(me * 4);
  L.tr = L.er1 + align256(me * 4);
  L.rslots = L.tr + align256(mt * 4);
  L.part = L.rslots + align256((size_t)(n + 1) * 4);
  // k-slice scratch per end: four partial results of the largest
  // intermediate, at most 8 Mi floats
  L.sk_floats = (size_t)std::min<int64_t>(4 * std::max(mt, me), 1ll << 23);
  L.sk = L.part + align256(kEnvDotParts * 8);
  L.skr = L.sk + align256(L.sk_floats * 4);
  L.total = L.skr + align256(L.sk_floats * 4);
  return L;
}

// ---------------------------------------------------------------------------
// MPO step kernels (contract the operator site with the T1 intermediate)

constexpr int kMaxW = 8;
constexpr int kMaxD = 4;

// left:  T2[a', t, v, b] = sum_{u, s} W[u, v, t, s] T1[a', u, s, b]
__global__ void __launch_bounds__(256) wstep_left_kernel(const float* __restrict__ t1, float* __restrict__ t2,
                                                         const float* __restrict__ w, int64_t w0, int64_t w1, int64_t w2,
                                                         int64_t w3, int da, int db, int wl, int wr, int d) {
  __shared__ float sw[kMaxW * kMaxW * kMaxD * kMaxD];
  const int nw = wl * wr * d * d;
  for (int i = threadIdx.x; i < nw; i += blockDim.x) {
    int s = i % d, t = (i / d) % d, v = (i / (d * d)) % wr, u = i / (d * d * wr);
    sw[i] = w[u * w0 + v * w1 + t * w2 + s * w3];
  }
  __syncthreads();
  const int64_t total = (int64_t)da * db;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total; idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t a = idx / db, b = idx - a * db;
    float x[kMaxW * kMaxD];
    for (int u = 0; u < wl; ++u)
      for (int s = 0; s < d; ++s) x[u * kMaxD + s] = t1[((a * wl + u) * d + s) * db + b];
    for (int t = 0; t < d; ++t)
      for (int v = 0; v < wr; ++v) {
        double acc = 0.0;
        for (int u = 0; u < wl; ++u)
          for (int s = 0; s < d; ++s) acc += (double)sw[((u * wr + v) * d + t) * d + s] * (double)x[u * kMaxD + s];
        t2[((a * d + t) * wr + v) * db + b] = (float)acc;
      }
  }
}

// right: T2'[u, a, t, b'] = sum_{s, v} W[u, v, t, s] T1'[a, s, b', v]
__global__ void __launch_bounds__(256) wstep_right_kernel(const float* __restrict__ t1, float* __restrict__ t2,
                                                          const float* __restrict__ w, int64_t w0, int64_t w1, int64_t w2,
                                                          int64_t w3, int da, int db, int wl, int wr, int d) {
  __shared__ float sw[kMaxW * kMaxW * kMaxD * kMaxD];
  const int nw = wl * wr * d * d;
  for (int i = threadIdx.x; i < nw; i += blockDim.x) {
    int s = i % d, t = (i / d) % d, v = (i / (d * d)) % wr, u = i / (d * d * wr);
    sw[i] = w[u * w0 + v * w1 + t * w2 + s * w3];
  }
  __syncthreads();
  const int64_t total = (int64_t)da * db;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total; idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t a = idx / db, b = idx - a * db;
    float x[kMaxD * kMaxW];
    for (int s = 0; s < d; ++s)
      for (int v = 0; v < wr; ++v) x[s * kMaxW + v] = t1[((a * d + s) * db + b) * wr + v];
    for (int u = 0; u < wl; ++u)
      for (int t = 0; t < d; ++t) {
        double acc = 0.0;
        for (int s = 0; s < d; ++s)
          for (int v = 0; v < wr; ++v) acc += (double)sw[((u * wr + v) * d + t) * d + s] * (double)x[s * kMaxW + v];
        t2[((u * (int64_t)da + a) * d + t) * db + b] = (float)acc;
      }
  }
}

// Specialised MPO steps for operator bonds WL, WR <= 5 and d = 2: one grid row
// per a (no index division), four consecutive b per thread (16-byte loads and
// stores), operand vectors held in registers.  Same FP64 accumulation.
typedef float f32x4w_t __attribute__((ext_vector_type(4)));

template <int WL, int WR, int D>
__global__ void __launch_bounds__(256) wstep_left_fixed(const float* __restrict__ t1, float* __restrict__ t2,
                                                        const float* __restrict__ w, int64_t w0, int64_t w1,
                                                        int64_t w2, int64_t w3, int db) {
  __shared__ float sw[WL * WR * D * D];
  for (int i = threadIdx.x; i < WL * WR * D * D; i += blockDim.x) {
    const int s = i % D, t = (i / D) % D, v = (i / (D * D)) % WR, u = i / (D * D * WR);
    sw[i] = w[u * w0 + v * w1 + t * w2 + s * w3];
  }
  __syncthreads();
  const int64_t a = blockIdx.y;
  const int b = (blockIdx.x * 256 + threadIdx.x) * 4;
  if (b >= db) return;
  f32x4w_t x[WL][D];
#pragma unroll
  for (int u = 0; u < WL; ++u)
#pragma unroll
    for (int s = 0; s < D; ++s) x[u][s] = *reinterpret_cast<const f32x4w_t*>(t1 + ((a * WL + u) * D + s) * db + b);
#pragma unroll
  for (int t = 0; t < D; ++t)
#pragma unroll
    for (int v = 0; v < WR; ++v) {
      double acc[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int u = 0; u < WL; ++u)
#pragma unroll
        for (int s = 0; s < D; ++s) {
          const double c = sw[((u * WR + v) * D + t) * D + s];
#pragma unroll
          for (int e = 0; e < 4; ++e) acc[e] += c * (double)x[u][s][e];
        }
      f32x4w_t o = {(float)acc[0], (float)acc[1], (float)acc[2], (float)acc[3]};
      *reinterpret_cast<f32x4w_t*>(t2 + ((a * D + t) * WR + v) * db + b) = o;
    }
}

template <int WL, int WR, int D>
__global__ void __launch_bounds__(256) wstep_right_fixed(const float* __restrict__ t1, float* __restrict__ t2,
                                                         const float* __restrict__ w, int64_t w0, int64_t w1,
                                                         int64_t w2, int64_t w3, int da, int db) {
  __shared__ float sw[WL * WR * D * D];
  for (int i = threadIdx.x; i < WL * WR * D * D; i += blockDim.x) {
    const int s = i % D, t = (i / D) % D, v = (i / (D * D)) % WR, u = i / (D * D * WR);
    sw[i] = w[u * w0 + v * w1 + t * w2 + s * w3];
  }
  __syncthreads();
  const int64_t a = blockIdx.y;
  const int b = (blockIdx.x * 256 + threadIdx.x) * 4;
  if (b >= db) return;
  // x[s][e * WR + v] = T1'[a, s, b + e, v]: 4 * WR consecutive floats per s
  float x[D][4 * WR];
#pragma unroll
  for (int s = 0; s < D; ++s) {
    const float* src = t1 + ((a * D + s) * db + b) * WR;
#pragma unroll
    for (int q = 0; q < WR; ++q) {
      const f32x4w_t y = *reinterpret_cast<const f32x4w_t*>(src + 4 * q);
#pragma unroll
      for (int e = 0; e < 4; ++e) x[s][4 * q + e] = y[e];
    }
  }
#pragma unroll
  for (int u = 0; u < WL; ++u)
#pragma unroll
    for (int t = 0; t < D; ++t) {
      double acc[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int s = 0; s < D; ++s)
#pragma unroll
        for (int v = 0; v < WR; ++v) {
          const double c = sw[((u * WR + v) * D + t) * D + s];
#pragma unroll
          for (int e = 0; e < 4; ++e) acc[e] += c * (double)x[s][e * WR + v];
        }
      f32x4w_t o = {(float)acc[0], (float)acc[1], (float)acc[2], (float)acc[3]};
      *reinterpret_cast<f32x4w_t*>(t2 + ((u * (int64_t)da + a) * D + t) * db + b) = o;
    }
}

// The left MPO step writing T2 with the pair (a', t) innermost: memory order
// [v, b, a', t], so the GEMM that contracts it with A_k over (a', t) reads
// that operand along k (16-byte loads, no transpose in registers).  A
// workgroup computes 16 a' x 64 b for every (t, v) from coalesced T1 rows,
// stages them in LDS (rows of 33 floats: conflict-free scalar writes) and
// writes each (v, b) row of 16 a' x 2 t as one 128-byte run.  Same FP64
// accumulation as the other steps.  Needs d = 2, da % 16 == 0, db % 64 == 0.
constexpr int kKmTa = 16, kKmTb = 64, kKmRow = kKmTa * 2 + 1;

template <int WL, int WR>
__global__ void __launch_bounds__(256) wstep_left_kmajor(const float* __restrict__ t1, float* __restrict__ t2,
                                                         const float* __restrict__ w, int64_t w0, int64_t w1,
                                                         int64_t w2, int64_t w3, int da, int db) {
  constexpr int D = 2;
  __shared__ float sw[WL * WR * D * D];
  __shared__ float tile[WR * kKmTb * kKmRow];
  for (int i = threadIdx.x; i < WL * WR * D * D; i += blockDim.x) {
    const int s = i % D, t = (i / D) % D, v = (i / (D * D)) % WR, u = i / (D * D * WR);
    sw[i] = w[u * w0 + v * w1 + t * w2 + s * w3];
  }
  __syncthreads();
  const int a0 = blockIdx.y * kKmTa, b0 = blockIdx.x * kKmTb;
  const int al = threadIdx.x / (kKmTb / 4), bq = threadIdx.x % (kKmTb / 4);
  const int64_t a = a0 + al;
  const int b = b0 + bq * 4;
  f32x4w_t x[WL][D];
#pragma unroll
  for (int u = 0; u < WL; ++u)
#pragma unroll
    for (int s = 0; s < D; ++s) x[u][s] = *reinterpret_cast<const f32x4w_t*>(t1 + ((a * WL + u) * D + s) * db + b);
#pragma unroll
  for (int t = 0; t < D; ++t)
#pragma unroll
    for (int v = 0; v < WR; ++v) {
      double acc[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int u = 0; u < WL; ++u)
#pragma unroll
        for (int s = 0; s < D; ++s) {
          const double c = sw[((u * WR + v) * D + t) * D + s];
#pragma unroll
          for (int e = 0; e < 4; ++e) acc[e] += c * (double)x[u][s][e];
        }
#pragma unroll
      for (int e = 0; e < 4; ++e) tile[(v * kKmTb + bq * 4 + e) * kKmRow + al * D + t] = (float)acc[e];
    }
  __syncthreads();
  // (v, b) rows of 32 floats; eight threads per row, four floats each
  for (int i = threadIdx.x; i < WR * kKmTb * 8; i += 256) {
    const int row = i / 8, c4 = (i % 8) * 4;
    const int v = row / kKmTb, bl = row % kKmTb;
    const float* src = tile + row * kKmRow + c4;
    const f32x4w_t o = {src[0], src[1], src[2], src[3]};
    *reinterpret_cast<f32x4w_t*>(t2 + (((int64_t)v * db + b0 + bl) * da + a0) * D + c4) = o;
  }
}

typedef void (*WstepKmFn)(const float*, float*, const float*, int64_t, int64_t, int64_t, int64_t, int, int);
template <int WL>
static WstepKmFn km_pick(int wr) {
  switch (wr) {
    case 1: return wstep_left_kmajor<WL, 1>;
    case 2: return wstep_left_kmajor<WL, 2>;
    case 3: return wstep_left_kmajor<WL, 3>;
    case 4: return wstep_left_kmajor<WL, 4>;
    case 5: return wstep_left_kmajor<WL, 5>;
    default: return nullptr;
  }
}
static WstepKmFn wstep_left_km_fn(int wl, int wr, int d, int64_t da, int64_t db, const void* t1, const void* t2) {
  if (d != 2 || da % kKmTa || db % kKmTb || reinterpret_cast<uintptr_t>(t1) % 16 || reinterpret_cast<uintptr_t>(t2) % 16)
    return nullptr;
  switch (wl) {
    case 1: return km_pick<1>(wr);
    case 2: return km_pick<2>(wr);
    case 3: return km_pick<3>(wr);
    case 4: return km_pick<4>(wr);
    case 5: return km_pick<5>(wr);
    default: return nullptr;
  }
}

typedef void (*WstepLeftFn)(const float*, float*, const float*, int64_t, int64_t, int64_t, int64_t, int);
typedef void (*WstepRightFn)(const float*, float*, const float*, int64_t, int64_t, int64_t, int64_t, int, int);

template <int WL>
static WstepLeftFn wl_pick(int wr) {
  switch (wr) {
    case 1: return wstep_left_fixed<WL, 1, 2>;
    case 2: return wstep_left_fixed<WL, 2, 2>;
    case 3: return wstep_left_fixed<WL, 3, 2>;
    case 4: return wstep_left_fixed<WL, 4, 2>;
    case 5: return wstep_left_fixed<WL, 5, 2>;
    default: return nullptr;
  }
}
template <int WL>
static WstepRightFn wr_pick(int wr) {
  switch (wr) {
    case 1: return wstep_right_fixed<WL, 1, 2>;
    case 2: return wstep_right_fixed<WL, 2, 2>;
    case 3: return wstep_right_fixed<WL, 3, 2>;
    case 4: return wstep_right_fixed<WL, 4, 2>;
    case 5: return wstep_right_fixed<WL, 5, 2>;
    default: return nullptr;
  }
}
// the specialised step for (wl, wr, d), or NULL when the shape needs the generic kernel
static WstepLeftFn wstep_left_fn(int wl, int wr, int d, int64_t db, const void* t1, const void* t2) {
  if (d != 2 || db % 4 || reinterpret_cast<uintptr_t>(t1) % 16 || reinterpret_cast<uintptr_t>(t2) % 16) return nullptr;
  switch (wl) {
    case 1: return wl_pick<1>(wr);
    case 2: return wl_pick<2>(wr);
    case 3: return wl_pick<3>(wr);
    case 4: return wl_pick<4>(wr);
    case 5: return wl_pick<5>(wr);
    default: return nullptr;
  }
}
static WstepRightFn wstep_right_fn(int wl, int wr, int d, int64_t db, const void* t1, const void* t2) {
  if (d != 2 || db % 4 || reinterpret_cast<uintptr_t>(t1) % 16 || reinterpret_cast<uintptr_t>(t2) % 16) return nullptr;
  switch (wl) {
    case 1: return wr_pick<1>(wr);
    case 2: return wr_pick<2>(wr);
    case 3: return wr_pick<3>(wr);
    case 4: return wr_pick<4>(wr);
    case 5: return wr_pick<5>(wr);
    default: return nullptr;
  }
}

__global__ void fill_one_kernel(float* p) { p[0] = 1.0f; }

__global__ void energy_kernel(const float* l_last, const float* r_first, double* e2) {
  if (threadIdx.x == 0) {
    e2[0] = l_last ? (double)l_last[0] : 0.0;
    e2[1] = r_first ? (double)r_first[0] : 0.0;
  }
}

static unsigned grid_for(int64_t n) {
  int64_t b = (n + 255) / 256;
  if (b > 8192) b = 8192;
  if (b < 1) b = 1;
  return (unsigned)b;
}

struct EnvLayout {
  size_t t1, t2, t1r, t2r, lbuf0, lbuf1, rbuf0, rbuf1, sk, skr, total;
  size_t sk_floats;   // k-slice partials per direction
};

// k-slice scratch per direction: four partial results of the largest site
// intermediate, at most 8 Mi floats (the GEMMs that k-slices help are the
// small ones)
constexpr int64_t kSliceScratchFloats = 1ll << 23;

static EnvLayout env_layout(int32_t n, const std::vector<int64_t>& dims, const std::vector<int64_t>& w, int64_t d) {
  int64_t mt = 1, me = 1;
  for (int k = 0; k < n; ++k) {
    mt = std::max(mt, dims[k] * w[k] * d * dims[k + 1]);      // T1 left, T2' right
    mt = std::max(mt, dims[k] * d * w[k + 1] * dims[k + 1]);  // T2 left, T1' right
  }
  for (int k = 0; k <= n; ++k) me = std::max(me, dims[k] * w[k] * dims[k]);
  EnvLayout L;
  // each direction has its own intermediates (the two sweeps may run concurrently)
  L.t1 = 0;
  L.t2 = align256(mt * 4);
  L.t1r = L.t2 + align256(mt * 4);
  L.t2r = L.t1r + align256(mt * 4);
  L.lbuf0 = L.t2r + align256(mt * 4);
  L.lbuf1 = L.lbuf0 + align256(me * 4);
  L.rbuf0 = L.lbuf1 + align256(me * 4);
  L.rbuf1 = L.rbuf0 + align256(me * 4);
  L.sk_floats = (size_t)std::min<int64_t>(4 * std::max(mt, me), kSliceScratchFloats);
  L.sk = L.rbuf1 + align256(me * 4);
  L.skr = L.sk + align256(L.sk_floats * 4);
  L.total = L.skr + align256(L.sk_floats * 4);
  return L;
}

// A second stream per device (default priority) on which the right sweep
// runs beside the left one; created on first use and kept for the process.
int32_t side_stream(hipStream_t& s) {
  constexpr int kPool = 4;
  struct DevPool {
    hipStream_t streams[kPool] = {};
    std::map<uintptr_t, int> slot_of;   // caller stream -> pool slot, assigned in turn
    int next = 0;
  };
  static std::mutex mu;
  static std::vector<DevPool> pools;
  int dev = 0;
  TN_TRY(hip_check(hipGetDevice(&dev), "get device"));
  std::lock_guard<std::mutex> lk(mu);
  if ((int)pools.size() <= dev) pools.resize(dev + 1);
  DevPool& P = pools[dev];
  const uintptr_t key = reinterpret_cast<uintptr_t>(s);
  auto it = P.slot_of.find(key);
  int slot;
  if (it != P.slot_of.end()) {
    slot = it->second;
  } else {
    slot = P.next;
    P.next = (P.next + 1) % kPool;
    P.slot_of[key] = slot;
  }
  if (!P.streams[slot])
    TN_TRY(hip_check(hipStreamCreateWithFlags(&P.streams[slot], hipStreamNonBlocking), "create stream"));
  s = P.streams[slot];
  return TN_OK;
}

static int32_t check_mpo(int32_t n, const tn_tensor* mpo, int64_t d, std::vector<int64_t>& w) {
  if (!mpo) return fail(TN_ERR_INVALID_ARGUMENT, "mpo is NULL");
  w.clear();
  for (int k = 0; k < n; ++k) {
    char nm[32];
    snprintf(nm, sizeof(nm), "mpo[%d]", k);
    TN_TRY(check_tensor(&mpo[k], nm, TN_F32));
    if (mpo[k].rank != 4) return fail(TN_ERR_SHAPE_MISMATCH, "%s must be [w_k, w_k+1, d, d]", nm);
    if (mpo[k].shape[2] != d || mpo[k].shape[3] != d) return fail(TN_ERR_SHAPE_MISMATCH, "%s: physical dims differ from the MPS", nm);
    if (k == 0) {
      if (mpo[0].shape[0] != 1) return fail(TN_ERR_SHAPE_MISMATCH, "mpo: first bond must be 1");
      w.push_back(1);
    } else if (mpo[k].shape[0] != w.back()) {
      return fail(TN_ERR_SHAPE_MISMATCH, "mpo: bond %d does not match", k);
    }
    if (mpo[k].shape[0] > kMaxW || mpo[k].shape[1] > kMaxW) return fail(TN_ERR_UNSUPPORTED, "MPO bond above %d", kMaxW);
    w.push_back(mpo[k].shape[1]);
  }
  if (w.back() != 1) return fail(TN_ERR_SHAPE_MISMATCH, "mpo: last bond must be 1");
  if (d > kMaxD) return fail(TN_ERR_UNSUPPORTED, "physical dimension above %d", kMaxD);
  return TN_OK;
}

static int32_t check_env_out(const tn_tensor* envs, int32_t n, const std::vector<int64_t>& dims,
                             const std::vector<int64_t>& w, const char* name) {
  if (!envs) return TN_OK;
  for (int k = 0; k <= n; ++k) {
    char nm[32];
    snprintf(nm, sizeof(nm), "%s[%d]", name, k);
    TN_TRY(check_tensor(&envs[k], nm, TN_F32));
    if (envs[k].rank != 3 || envs[k].shape[0] != dims[k] || envs[k].shape[1] != w[k] || envs[k].shape[2] != dims[k])
      return fail(TN_ERR_SHAPE_MISMATCH, "%s must be [D_k, w_k, D_k]", nm);
    if (has_internal_overlap(envs[k])) return fail(TN_ERR_INVALID_ARGUMENT, "%s maps two indices to one address", nm);
  }
  return TN_OK;
}

}  // namespace tn

using namespace tn;

extern "C" {

int32_t tn_mps_inner_workspace(int32_t n_sites, const tn_tensor* psi, const tn_tensor* phi, size_t* bytes) {
  if (!bytes) return fail(TN_ERR_INVALID_ARGUMENT, "bytes is NULL");
  std::vector<int64_t> dp, dq;
  int64_t d1 = 0, d2 = 0;
  TN_TRY(check_chain(n_sites, psi, "psi", TN_F32, &dp, &d1));
  TN_TRY(check_chain(n_sites, phi, "phi", TN_F32, &dq, &d2));
  if (d1 != d2) return fail(TN_ERR_SHAPE_MISMATCH, "psi and phi have different physical dimensions");
  *bytes = inner_layout(n_sites, dp, dq, d1).total;
  return TN_OK;
}

int32_t tn_mps_inner(int32_t n_sites, const tn_tensor* psi, const tn_tensor* phi, double* out2, void* workspace,
                     size_t ws_bytes, int32_t prec, void* stream) {
  std::vector<int64_t> dp, dq;
  int64_t d1 = 0, d2 = 0;
  TN_TRY(check_chain(n_sites, psi, "psi", TN_F32, &dp, &d1));
  TN_TRY(check_chain(n_sites, phi, "phi", TN_F32, &dq, &d2));
  if (d1 != d2) return fail(TN_ERR_SHAPE_MISMATCH, "psi and phi have different physical dimensions");
  if (!out2) return fail(TN_ERR_INVALID_ARGUMENT, "out2 is NULL");
  if (prec < 0 || prec > 3) return fail(TN_ERR_UNSUPPORTED, "unknown precision %d", prec);
  InnerLayout L = inner_layout(n_sites, dp, dq, d1);
  if (ws_bytes < L.total || !workspace) return fail(TN_ERR_WORKSPACE_TOO_SMALL, "workspace needs %zu bytes", L.total);
  hipStream_t st = static_cast<hipStream_t>(stream);
  char* ws = static_cast<char*>(workspace);
  float* e[2] = {reinterpret_cast<float*>(ws + L.e0), reinterpret_cast<float*>(ws + L.e1)};
  float* t = reinterpret_cast<float*>(ws + L.t);
  uint32_t* slots = reinterpret_cast<uint32_t*>(ws + L.slots);
  float* sk = reinterpret_cast<float*>(ws + L.sk);
  float* skr = reinterpret_cast<float*>(ws + L.skr);
  if (n_sites < kInnerTwoSided) {
    hipLaunchKernelGGL(mps_init_kernel, dim3(grid_for(n_sites + 1)), dim3(256), 0, st, e[0], slots, n_sites + 1);
    TN_TRY(hip_check(hipGetLastError(), "mps init"));
    for (int k = 0; k < n_sites; ++k)
      TN_TRY(inner_site(psi[k], phi[k], e[k & 1], e[(k + 1) & 1], t, slots, k, prec, st, sk, L.sk_floats));
    hipLaunchKernelGGL(mps_finish_kernel, dim3(1), dim3(256), 0, st, e[n_sites & 1], slots, n_sites, out2);
    return hip_check(hipGetLastError(), "mps finish");
  }
  // Two-sided: sites 0 .. c-1 from the left on the caller's stream, sites
  // n-1 .. c from the right on a side stream forked from it and joined back
  // (capturable), issued site by site so both streams always have work.
  // Each half is a chain of dependent GEMMs that alone leaves most of the
  // chip idle at chi <= 1024; the two halves overlap.
  const int c = n_sites / 2, nr = n_sites - c;
  float* er[2] = {reinterpret_cast<float*>(ws + L.er0), reinterpret_cast<float*>(ws + L.er1)};
  float* tr = reinterpret_cast<float*>(ws + L.tr);
  uint32_t* rslots = reinterpret_cast<uint32_t*>(ws + L.rslots);   // rslots[i]: E_R at bond n - i
  double* part = reinterpret_cast<double*>(ws + L.part);
  hipStream_t rs = st;
  TN_TRY(side_stream(rs));
  hipEvent_t fork = nullptr, join = nullptr;
  TN_TRY(hip_check(hipEventCreateWithFlags(&fork, hipEventDisableTiming), "create event"));
  if (hipEventCreateWithFlags(&join, hipEventDisableTiming) != hipSuccess) {
    hipEventDestroy(fork);
    return fail(TN_ERR_DEVICE, "create event failed");
  }
  hipEventRecord(fork, st);
  hipStreamWaitEvent(rs, fork, 0);
  hipLaunchKernelGGL(mps_init_kernel, dim3(grid_for(c + 1)), dim3(256), 0, st, e[0], slots, c + 1);
  hipLaunchKernelGGL(mps_init_kernel, dim3(grid_for(nr + 1)), dim3(256), 0, rs, er[0], rslots, nr + 1);
  int32_t rc = hip_check(hipGetLastError(), "mps init");
  {
    SharedChipScope shared;
    for (int i = 0; i < std::max(c, nr) && rc == TN_OK; ++i) {
      if (i < c) rc = inner_site(psi[i], phi[i], e[i & 1], e[(i + 1) & 1], t, slots, i, prec, st, sk, L.sk_floats);
      if (rc == TN_OK && i < nr) {
        const int k = n_sites - 1 - i;
        rc = inner_site_right(psi[k], phi[k], er[i & 1], er[(i + 1) & 1], tr, rslots + i, rslots + i + 1, prec, rs,
                              skr, L.sk_floats);
      }
    }
  }
  hipEventRecord(join, rs);
  hipStreamWaitEvent(st, join, 0);
  hipEventDestroy(fork);
  hipEventDestroy(join);
  TN_TRY(rc);
  const int64_t cnt = dp[c] * dq[c];
  const int64_t parts = std::min<int64_t>(kEnvDotParts, (cnt + 255) / 256);
  hipLaunchKernelGGL(env_dot_partial_kernel, dim3((unsigned)parts), dim3(256), 0, st, e[c & 1], er[nr & 1], cnt, part);
  hipLaunchKernelGGL(env_dot_finish_kernel, dim3(1), dim3(256), 0, st, part, (int)parts, slots, c, rslots, nr, out2);
  return hip_check(hipGetLastError(), "mps finish");
}

// ----------------------------------------------------------------------------
// uneven batch

int32_t tn_mps_inner_batched_workspace(int32_t n_chains, const int32_t* site_offsets, const tn_tensor* psi_sites,
                                       const tn_tensor* phi_sites, size_t* bytes);
int32_t tn_mps_inner_batched(int32_t n_chains, const int32_t* site_offsets, const tn_tensor* psi_sites,
                             const tn_tensor* phi_sites, double* out2, void* workspace, size_t ws_bytes, int32_t prec,
                             void* stream);

// ----------------------------------------------------------------------------
// environment sweep

int32_t tn_mps_env_sweep_workspace(int32_t n_sites, const tn_tensor* psi, const tn_tensor* mpo, size_t* bytes) {
  if (!bytes) return fail(TN_ERR_INVALID_ARGUMENT, "bytes is NULL");
  std::vector<int64_t> dims, w;
  int64_t d = 0;
  TN_TRY(check_chain(n_sites, psi, "psi", TN_F32, &dims, &d));
  TN_TRY(check_mpo(n_sites, mpo, d, w));
  *bytes = env_layout(n_sites, dims, w, d).total;
  return TN_OK;
}

int32_t tn_mps_env_sweep(int32_t n_sites, const tn_tensor* psi, const tn_tensor* mpo, tn_tensor* L_out,
                         tn_tensor* R_out, double* energy2, int32_t which, void* workspace, size_t ws_bytes, int32_t prec,
                         void* stream) {
  std::vector<int64_t> dims, w;
  int64_t d = 0;
  TN_TRY(check_chain(n_sites, psi, "psi", TN_F32, &dims, &d));
  TN_TRY(check_mpo(n_sites, mpo, d, w));
  TN_TRY(check_env_out(L_out, n_sites, dims, w, "L_out"));
  TN_TRY(check_env_out(R_out, n_sites, dims, w, "R_out"));
  if (which < 1 || which > 3) return fail(TN_ERR_INVALID_ARGUMENT, "which must be 1 (left), 2 (right) or 3");
  if (prec < 0 || prec > 3) return fail(TN_ERR_UNSUPPORTED, "unknown precision %d", prec);
  for (int k = 0; k < n_sites; ++k)
    if (dims[k] * std::max(w[k], w[k + 1]) * d * dims[k + 1] >= (1ll << 31))
      return fail(TN_ERR_UNSUPPORTED, "site %d intermediate larger than 2^31 elements", k);
  EnvLayout L = env_layout(n_sites, dims, w, d);
  if (ws_bytes < L.total || !workspace) return fail(TN_ERR_WORKSPACE_TOO_SMALL, "workspace needs %zu bytes", L.total);
  hipStream_t st = static_cast<hipStream_t>(stream);
  char* ws = static_cast<char*>(workspace);
  float* t1 = reinterpret_cast<float*>(ws + L.t1);
  float* t2 = reinterpret_cast<float*>(ws + L.t2);
  float* t1r = reinterpret_cast<float*>(ws + L.t1r);
  float* t2r = reinterpret_cast<float*>(ws + L.t2r);
  float* buf[2] = {reinterpret_cast<float*>(ws + L.lbuf0), reinterpret_cast<float*>(ws + L.lbuf1)};
  float* rbuf[2] = {reinterpret_cast<float*>(ws + L.rbuf0), reinterpret_cast<float*>(ws + L.rbuf1)};
  float* skl = reinterpret_cast<float*>(ws + L.sk);
  float* skr = reinterpret_cast<float*>(ws + L.skr);

  // left site k: L_k -> T1 -> (MPO step) T2 -> L_{k+1}
  auto left_site = [&](int k, tn_tensor& cur, hipStream_t s) -> int32_t {
    SplitKScope slices(skl, L.sk_floats);
    const int64_t da = dims[k], db = dims[k + 1], wl = w[k], wr = w[k + 1];
    tn_tensor T1 = make_view(t1, TN_F32, {da, wl, d, db});
    tn_tensor T2 = make_view(t2, TN_F32, {da, d, wr, db});
    tn_tensor nxt = L_out ? L_out[k + 1] : make_view(buf[(k + 1) & 1], TN_F32, {db, wr, db});
    GemmDesc g;
    const int32_t a1[1] = {2}, b1[1] = {0};
    TN_TRY(plan_gemm(cur, psi[k], 1, a1, b1, T1, g));
    TN_TRY(launch_gemm(g, prec, s));
    const tn_tensor& W = mpo[k];
    const int32_t a3[2] = {0, 1}, b3[2] = {0, 1};
    if (WstepKmFn f = wstep_left_km_fn((int)wl, (int)wr, (int)d, da, db, t1, t2)) {
      // T2 in memory order [v, b, a', t]: the view keeps the axis order (a', t, v, b)
      hipLaunchKernelGGL(f, dim3((unsigned)(db / kKmTb), (unsigned)(da / kKmTa)), dim3(256), 0, s, t1, t2,
                         static_cast<const float*>(W.data), W.stride[0], W.stride[1], W.stride[2], W.stride[3], (int)da,
                         (int)db);
      TN_TRY(hip_check(hipGetLastError(), "wstep left"));
      tn_tensor T2k = T2;
      T2k.stride[0] = d;
      T2k.stride[1] = 1;
      T2k.stride[2] = db * da * d;
      T2k.stride[3] = da * d;
      TN_TRY(plan_gemm(psi[k], T2k, 2, a3, b3, nxt, g));
      TN_TRY(launch_gemm(g, prec, s));
      cur = nxt;
      return TN_OK;
    }
    if (WstepLeftFn f = wstep_left_fn((int)wl, (int)wr, (int)d, db, t1, t2))
      hipLaunchKernelGGL(f, dim3((unsigned)((db / 4 + 255) / 256), (unsigned)da), dim3(256), 0, s, t1, t2,
                         static_cast<const float*>(W.data), W.stride[0], W.stride[1], W.stride[2], W.stride[3], (int)db);
    else
      hipLaunchKernelGGL(wstep_left_kernel, dim3(grid_for(da * db)), dim3(256), 0, s, t1, t2,
                         static_cast<const float*>(W.data), W.stride[0], W.stride[1], W.stride[2], W.stride[3], (int)da,
                         (int)db, (int)wl, (int)wr, (int)d);
    TN_TRY(hip_check(hipGetLastError(), "wstep left"));
    TN_TRY(plan_gemm(psi[k], T2, 2, a3, b3, nxt, g));
    TN_TRY(launch_gemm(g, prec, s));
    cur = nxt;
    return TN_OK;
  };
  // right site k: R_{k+1} -> T1' -> (MPO step) T2' -> R_k
  auto right_site = [&](int k, tn_tensor& cur, hipStream_t s) -> int32_t {
    SplitKScope slices(skr, L.sk_floats);
    const int64_t da = dims[k], db = dims[k + 1], wl = w[k], wr = w[k + 1];
    tn_tensor T1 = make_view(t1r, TN_F32, {da, d, db, wr});
    tn_tensor T2 = make_view(t2r, TN_F32, {wl, da, d, db});
    tn_tensor nxt = R_out ? R_out[k] : make_view(rbuf[k & 1], TN_F32, {da, wl, da});
    GemmDesc g;
    const int32_t a1[1] = {2}, b1[1] = {2};
    TN_TRY(plan_gemm(psi[k], cur, 1, a1, b1, T1, g));
    TN_TRY(launch_gemm(g, prec, s));
    const tn_tensor& W = mpo[k];
    if (WstepRightFn f = wstep_right_fn((int)wl, (int)wr, (int)d, db, t1r, t2r))
      hipLaunchKernelGGL(f, dim3((unsigned)((db / 4 + 255) / 256), (unsigned)da), dim3(256), 0, s, t1r, t2r,
                         static_cast<const float*>(W.data), W.stride[0], W.stride[1], W.stride[2], W.stride[3], (int)da,
                         (int)db);
    else
      hipLaunchKernelGGL(wstep_right_kernel, dim3(grid_for(da * db)), dim3(256), 0, s, t1r, t2r,
                         static_cast<const float*>(W.data), W.stride[0], W.stride[1], W.stride[2], W.stride[3], (int)da,
                         (int)db, (int)wl, (int)wr, (int)d);
    TN_TRY(hip_check(hipGetLastError(), "wstep right"));
    const int32_t a3[2] = {1, 2}, b3[2] = {2, 3};
    TN_TRY(plan_gemm(psi[k], T2, 2, a3, b3, nxt, g));
    TN_TRY(launch_gemm(g, prec, s));
    cur = nxt;
    return TN_OK;
  };

  // Both directions: the right sweep runs on a side stream forked from and
  // joined back into the caller's stream (capturable), and the two are
  // issued site by site so both streams always have work queued.
  hipStream_t rs = st;
  hipEvent_t fork = nullptr, join = nullptr;
  if (which == 3) {
    TN_TRY(side_stream(rs));
    TN_TRY(hip_check(hipEventCreateWithFlags(&fork, hipEventDisableTiming), "create event"));
    if (hipEventCreateWithFlags(&join, hipEventDisableTiming) != hipSuccess) {
      hipEventDestroy(fork);
      return fail(TN_ERR_DEVICE, "create event failed");
    }
    hipEventRecord(fork, st);
    hipStreamWaitEvent(rs, fork, 0);
  }
  tn_tensor lcur, rcur;
  if (which & 1) {
    lcur = L_out ? L_out[0] : make_view(buf[0], TN_F32, {1, 1, 1});
    hipLaunchKernelGGL(fill_one_kernel, dim3(1), dim3(1), 0, st, static_cast<float*>(lcur.data));
  }
  if (which & 2) {
    rcur = R_out ? R_out[n_sites] : make_view(rbuf[n_sites & 1], TN_F32, {1, 1, 1});
    hipLaunchKernelGGL(fill_one_kernel, dim3(1), dim3(1), 0, rs, static_cast<float*>(rcur.data));
  }
  int32_t rc = TN_OK;
  {
    SharedChipScope shared(which == 3);
    for (int i = 0; i < n_sites && rc == TN_OK; ++i) {
      if (which & 1) rc = left_site(i, lcur, st);
      if (rc == TN_OK && (which & 2)) rc = right_site(n_sites - 1 - i, rcur, rs);
    }
  }
  if (which == 3) {
    hipEventRecord(join, rs);
    hipStreamWaitEvent(st, join, 0);
    hipEventDestroy(fork);
    hipEventDestroy(join);
  }
  TN_TRY(rc);
  const float* l_last = (which & 1) ? static_cast<const float*>(lcur.data) : nullptr;
  const float* r_first = (which & 2) ? static_cast<const float*>(rcur.data) : nullptr;
  if (energy2) {
    hipLaunchKernelGGL(energy_kernel, dim3(1), dim3(64), 0, st, l_last, r_first, energy2);
    TN_TRY(hip_check(hipGetLastError(), "energy"));
  }
  return TN_OK;
}

}  // extern "C"
