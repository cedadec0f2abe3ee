// Complex contractions (the V^dagger of section III.B: complex nodes with
// conjugation) on the real contraction kernels.
//
// A complex tensor (TN_C64) is interleaved (real, imaginary) float pairs, so
// A viewed as a real tensor gains an innermost axis ri of extent 2.  The
// right operand is expanded once into a real tensor
//     B'[k..., ri, n..., ro]  with  B'[ri=0, ro=0] =  Re B,   B'[ri=1, ro=0] = -sa Im' B,
//                                   B'[ri=0, ro=1] =  Im' B,  B'[ri=1, ro=1] =  sa Re B,
// (Im' B = sb Im B; sa, sb = -1 when A, B are conjugated), laid out with the
// contracted axes and ri as one block and the free axes and ro as another,
// so that
//     C[free_a..., free_b..., ro] = sum_{k, ri} A[..., k, ..., ri] B'[k..., ri, free_b..., ro]
// is one real contraction over the merged (k, ri) index: the real and
// imaginary parts of the complex products (four real products each) come
// out interleaved, i.e. as the complex output itself.  Every precision of
// the real path applies, the split-BF16 products included.
#include <cmath>
#include <cstring>
#include <vector>

#include "internal.h"

namespace tn {

namespace {

struct ExpandArgs {
  const float* b;          // interleaved complex
  float* bx;               // expanded real operand
  int32_t rank;
  int64_t shape[TN_MAX_RANK];
  int64_t stride[TN_MAX_RANK];   // complex elements
  int64_t xstride[TN_MAX_RANK];  // floats in bx
  int64_t ri_stride;             // floats
  int64_t total;
  float sa, sb;
};

__global__ void expand_kernel(ExpandArgs e) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < e.total; i += (int64_t)gridDim.x * blockDim.x) {
    int64_t idx = i, src = 0, dst = 0;
    for (int a = e.rank - 1; a >= 0; --a) {
      const int64_t q = idx / e.shape[a], r = idx - q * e.shape[a];
      src += r * e.stride[a];
      dst += r * e.xstride[a];
      idx = q;
    }
    const float re = e.b[2 * src], im = e.sb * e.b[2 * src + 1];
    e.bx[dst] = re;                               // ri 0, ro 0
    e.bx[dst + 1] = im;                           // ri 0, ro 1
    e.bx[dst + e.ri_stride] = -e.sa * im;         // ri 1, ro 0
    e.bx[dst + e.ri_stride + 1] = e.sa * re;      // ri 1, ro 1
  }
}

// real view of a complex tensor with the ri (or ro) axis appended
tn_tensor real_view(const tn_tensor& t) {
  tn_tensor v = t;
  v.dtype = TN_F32;
  for (int i = 0; i < t.rank; ++i) v.stride[i] = 2 * t.stride[i];
  v.shape[t.rank] = 2;
  v.stride[t.rank] = 1;
  v.rank = t.rank + 1;
  return v;
}

size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

int32_t check_c64(const tn_tensor* t, const char* name, int max_rank) {
  TN_TRY(check_tensor(t, name, TN_C64));
  if (t->rank > max_rank) return fail(TN_ERR_UNSUPPORTED, "%s: complex rank above %d", name, max_rank);
  return TN_OK;
}

}  // namespace

size_t c64_workspace_bytes(const tn_tensor& b) { return al256((size_t)numel(b) * 16) + kReduceScratchBytes; }

int32_t contract_c64_impl(const tn_tensor* a, const tn_tensor* b, int32_t n_pairs, const int32_t* axes_a,
                          const int32_t* axes_b, int conj_a, int conj_b, tn_tensor* out, void* workspace,
                          size_t ws_bytes, int32_t prec, hipStream_t st) {
  TN_TRY(check_c64(a, "a", TN_MAX_RANK - 1));
  TN_TRY(check_c64(b, "b", TN_MAX_RANK - 2));
  TN_TRY(check_c64(out, "out", TN_MAX_RANK - 1));
  if (n_pairs < 0 || n_pairs > std::min(a->rank, b->rank)) return fail(TN_ERR_INVALID_ARGUMENT, "bad pair count %d", n_pairs);
  if (n_pairs > 0 && (!axes_a || !axes_b)) return fail(TN_ERR_INVALID_ARGUMENT, "axes are NULL");
  std::vector<int> used_a(a->rank, 0), used_b(b->rank, 0);
  for (int p = 0; p < n_pairs; ++p) {
    const int i = axes_a[p], j = axes_b[p];
    if (i < 0 || i >= a->rank || j < 0 || j >= b->rank || used_a[i] || used_b[j])
      return fail(TN_ERR_INVALID_ARGUMENT, "pair %d: axes (%d, %d) out of range or repeated", p, i, j);
    if (a->shape[i] != b->shape[j]) return fail(TN_ERR_SHAPE_MISMATCH, "pair %d: dimensions %lld and %lld differ", p,
                                                (long long)a->shape[i], (long long)b->shape[j]);
    used_a[i] = used_b[j] = 1;
  }
  const size_t need = c64_workspace_bytes(*b);
  if (!workspace || ws_bytes < need) return fail(TN_ERR_WORKSPACE_TOO_SMALL, "workspace needs %zu bytes", need);
  if (overlaps(*out, *a) || overlaps(*out, *b)) return fail(TN_ERR_ALIASING, "out overlaps an input");
  {
    tn_tensor wsv = make_view(workspace, TN_F32, {(int64_t)(need / 4)});
    if (overlaps(*out, wsv) || overlaps(*a, wsv) || overlaps(*b, wsv))
      return fail(TN_ERR_ALIASING, "the workspace overlaps a tensor");
  }
  // B' layout: [contracted axes in pair order][ri][free axes in order][ro]
  std::vector<int> free_b;
  for (int j = 0; j < b->rank; ++j)
    if (!used_b[j]) free_b.push_back(j);
  int64_t nfree = 1;
  for (int j : free_b) nfree *= b->shape[j];
  ExpandArgs e;
  std::memset(&e, 0, sizeof(e));
  e.b = static_cast<const float*>(b->data);
  e.bx = static_cast<float*>(workspace);
  e.rank = b->rank;
  e.total = numel(*b);
  e.sa = conj_a ? -1.f : 1.f;
  e.sb = conj_b ? -1.f : 1.f;
  e.ri_stride = nfree * 2;
  for (int j = 0; j < b->rank; ++j) {
    e.shape[j] = b->shape[j];
    e.stride[j] = b->stride[j];
  }
  int64_t acc = 2;   // ro
  for (int q = (int)free_b.size() - 1; q >= 0; --q) {
    e.xstride[free_b[q]] = acc;
    acc *= b->shape[free_b[q]];
  }
  acc *= 2;          // ri
  for (int p = n_pairs - 1; p >= 0; --p) {
    e.xstride[axes_b[p]] = acc;
    acc *= b->shape[axes_b[p]];
  }
  hipLaunchKernelGGL(expand_kernel, dim3((unsigned)std::max<int64_t>(1, std::min<int64_t>((e.total + 255) / 256, 16384))),
                     dim3(256), 0, st, e);
  TN_TRY(hip_check(hipGetLastError(), "complex expand"));
  tn_tensor ar = real_view(*a), orv = real_view(*out);
  tn_tensor br;
  std::memset(&br, 0, sizeof(br));
  br.data = workspace;
  br.dtype = TN_F32;
  br.rank = b->rank + 2;
  for (int j = 0; j < b->rank; ++j) {
    br.shape[j] = b->shape[j];
    br.stride[j] = e.xstride[j];
  }
  br.shape[b->rank] = 2;           // ri
  br.stride[b->rank] = e.ri_stride;
  br.shape[b->rank + 1] = 2;       // ro
  br.stride[b->rank + 1] = 1;
  std::vector<int32_t> pa(axes_a, axes_a + n_pairs), pb(axes_b, axes_b + n_pairs);
  pa.push_back(a->rank);
  pb.push_back(b->rank);
  void* scratch = static_cast<char*>(workspace) + al256((size_t)numel(*b) * 16);
  return contract_between_impl(&ar, &br, n_pairs + 1, pa.data(), pb.data(), &orv, scratch, kReduceScratchBytes, prec, st);
}

namespace {

// ---------------------------------------------------------------------------
// complex MPS inner product

__global__ void c64_init_kernel(float* e, unsigned* slot, double* acc) {
  e[0] = 1.f;
  e[1] = 0.f;
  slot[0] = 0u;
  acc[0] = 0.0;
}

__global__ void zero_u32_kernel(unsigned* p) { p[0] = 0u; }

// slot = max over the n complex entries of max(|re|, |im|) (as float bits)
__global__ void c64_absmax_kernel(const float* e, int64_t n, unsigned* slot) {
  __shared__ float red[256];
  float m = 0.f;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < 2 * n; i += (int64_t)gridDim.x * blockDim.x)
    m = fmaxf(m, fabsf(e[i]));
  red[threadIdx.x] = m;
  __syncthreads();
  for (int o = 128; o >= 1; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + o]);
    __syncthreads();
  }
  if (threadIdx.x == 0) atomicMax(slot, __float_as_uint(red[0]));
}

// e *= 2^-x with x the binary exponent of the slot's maximum (exact); acc += x
__global__ void c64_rescale_kernel(float* e, int64_t n, const unsigned* slot, double* acc) {
  const float mx = __uint_as_float(slot[0]);
  int x = 0;
  if (mx > 0.f && isfinite(mx)) frexpf(mx, &x);
  const float sc = ldexpf(1.f, -x);
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < 2 * n; i += (int64_t)gridDim.x * blockDim.x)
    e[i] *= sc;
  if (blockIdx.x == 0 && threadIdx.x == 0) acc[0] += (double)x;
}

__global__ void c64_finish_kernel(const float* e, const double* acc, double* out4) {
  out4[0] = (double)e[0];
  out4[1] = (double)e[1];
  out4[2] = acc[0] * 0.6931471805599453;
  out4[3] = 0.0;
}

struct C64InnerLayout {
  size_t e0, e1, t, ctl, x, total;
  int64_t me, mt, mx;
};

int32_t c64_inner_layout(int32_t n, const tn_tensor* psi, const tn_tensor* phi, C64InnerLayout& L) {
  if (n < 1 || !psi || !phi) return fail(TN_ERR_INVALID_ARGUMENT, "need n_sites >= 1 and both chains");
  L.me = L.mt = L.mx = 1;
  int64_t dp = 1, dq = 1;
  for (int k = 0; k < n; ++k) {
    char nm[32];
    snprintf(nm, sizeof(nm), "psi[%d]", k);
    TN_TRY(check_c64(&psi[k], nm, 3));
    snprintf(nm, sizeof(nm), "phi[%d]", k);
    TN_TRY(check_c64(&phi[k], nm, 3));
    if (psi[k].rank != 3 || phi[k].rank != 3) return fail(TN_ERR_SHAPE_MISMATCH, "sites must be [D_k, d, D_k+1]");
    if (psi[k].shape[0] != dp || phi[k].shape[0] != dq) return fail(TN_ERR_SHAPE_MISMATCH, "site %d: left bond differs", k);
    if (psi[k].shape[1] != phi[k].shape[1]) return fail(TN_ERR_SHAPE_MISMATCH, "site %d: physical dims differ", k);
    const int64_t t = dp * psi[k].shape[1] * phi[k].shape[2];
    L.mt = std::max(L.mt, t);
    dp = psi[k].shape[2];
    dq = phi[k].shape[2];
    L.me = std::max(L.me, dp * dq);
    L.mx = std::max(L.mx, std::max(numel(phi[k]), t));
  }
  if (dp != 1 || dq != 1) return fail(TN_ERR_SHAPE_MISMATCH, "the last bond must be 1");
  size_t o = 0;
  L.e0 = o;
  o += al256((size_t)L.me * 8);
  L.e1 = o;
  o += al256((size_t)L.me * 8);
  L.t = o;
  o += al256((size_t)L.mt * 8);
  L.ctl = o;
  o += 256;
  L.x = o;
  o += al256((size_t)L.mx * 16) + kReduceScratchBytes;
  L.total = o;
  return TN_OK;
}

}  // namespace

}  // namespace tn

using namespace tn;

extern "C" {

int32_t tn_contract_between_c64_workspace(const tn_tensor* b, size_t* bytes) {
  if (!bytes) return fail(TN_ERR_INVALID_ARGUMENT, "bytes is NULL");
  TN_TRY(check_c64(b, "b", TN_MAX_RANK - 2));
  *bytes = c64_workspace_bytes(*b);
  return TN_OK;
}

int32_t tn_contract_between_c64(const tn_tensor* a, const tn_tensor* b, int32_t n_pairs, const int32_t* axes_a,
                                const int32_t* axes_b, int32_t conj_a, int32_t conj_b, tn_tensor* out, void* workspace,
                                size_t ws_bytes, int32_t prec, void* stream) {
  if (prec < 0 || prec > 3) return fail(TN_ERR_UNSUPPORTED, "unknown precision %d", prec);
  return contract_c64_impl(a, b, n_pairs, axes_a, axes_b, conj_a != 0, conj_b != 0, out, workspace, ws_bytes, prec,
                           static_cast<hipStream_t>(stream));
}

int32_t tn_mps_inner_c64_workspace(int32_t n_sites, const tn_tensor* psi, const tn_tensor* phi, size_t* bytes) {
  if (!bytes) return fail(TN_ERR_INVALID_ARGUMENT, "bytes is NULL");
  C64InnerLayout L;
  TN_TRY(c64_inner_layout(n_sites, psi, phi, L));
  *bytes = L.total;
  return TN_OK;
}

int32_t tn_mps_inner_c64(int32_t n_sites, const tn_tensor* psi, const tn_tensor* phi, double* out4, void* workspace,
                         size_t ws_bytes, int32_t prec, void* stream) {
  C64InnerLayout L;
  TN_TRY(c64_inner_layout(n_sites, psi, phi, L));
  if (!out4) return fail(TN_ERR_INVALID_ARGUMENT, "out4 is NULL");
  if (prec < 0 || prec > 3) return fail(TN_ERR_UNSUPPORTED, "unknown precision %d", prec);
  if (!workspace || ws_bytes < L.total) return fail(TN_ERR_WORKSPACE_TOO_SMALL, "workspace needs %zu bytes", L.total);
  hipStream_t st = static_cast<hipStream_t>(stream);
  char* ws = static_cast<char*>(workspace);
  float* e[2] = {reinterpret_cast<float*>(ws + L.e0), reinterpret_cast<float*>(ws + L.e1)};
  float* t = reinterpret_cast<float*>(ws + L.t);
  unsigned* slot = reinterpret_cast<unsigned*>(ws + L.ctl);
  double* acc = reinterpret_cast<double*>(ws + L.ctl + 8);
  void* xws = ws + L.x;
  const size_t xbytes = L.total - L.x;
  hipLaunchKernelGGL(c64_init_kernel, dim3(1), dim3(1), 0, st, e[0], slot, acc);
  int64_t dp = 1, dq = 1;
  for (int k = 0; k < n_sites; ++k) {
    const int64_t d = psi[k].shape[1], dp1 = psi[k].shape[2], dq1 = phi[k].shape[2];
    tn_tensor ev = make_view(e[k & 1], TN_C64, {dp, dq});
    tn_tensor tv = make_view(t, TN_C64, {dp, d, dq1});
    tn_tensor en = make_view(e[(k + 1) & 1], TN_C64, {dp1, dq1});
    const int32_t p0[1] = {1}, q0[1] = {0};
    TN_TRY(contract_c64_impl(&ev, &phi[k], 1, p0, q0, 0, 0, &tv, xws, xbytes, prec, st));   // T = E . phi_k
    const int32_t p1[2] = {0, 1}, q1[2] = {0, 1};
    TN_TRY(contract_c64_impl(&psi[k], &tv, 2, p1, q1, 1, 0, &en, xws, xbytes, prec, st));  // E' = psi_k^* . T
    const int64_t ne = dp1 * dq1;
    const unsigned blocks = (unsigned)std::max<int64_t>(1, std::min<int64_t>((2 * ne + 255) / 256, 1024));
    hipLaunchKernelGGL(zero_u32_kernel, dim3(1), dim3(1), 0, st, slot);
    hipLaunchKernelGGL(c64_absmax_kernel, dim3(blocks), dim3(256), 0, st, e[(k + 1) & 1], ne, slot);
    hipLaunchKernelGGL(c64_rescale_kernel, dim3(blocks), dim3(256), 0, st, e[(k + 1) & 1], ne, slot, acc);
    dp = dp1;
    dq = dq1;
  }
  hipLaunchKernelGGL(c64_finish_kernel, dim3(1), dim3(1), 0, st, e[n_sites & 1], acc, out4);
  return hip_check(hipGetLastError(), "complex inner product");
}

}  // extern "C"
