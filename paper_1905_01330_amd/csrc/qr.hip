// Left-canonical gauge of an MPS in FP64 on the GPU: successive Householder
// QR factorisations (Golub and Van Loan, "Matrix Computations", 5.1-5.2).
// For site k the carried triangular factor is absorbed first
// (X = R_{k-1} A_k viewed as (D_k d) x D_{k+1}), X is factorised in place
// column by column (one reflector kernel and one trailing-update kernel per
// column), the thin Q is accumulated backwards from [I; 0], and signs are
// fixed so that diag(R) >= 0.  X and Q are kept column-major so every
// reflector and column update reads contiguous memory.
#include <algorithm>
#include <cmath>
#include <vector>

#include "internal.h"

namespace tn {

static size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

__device__ inline double block_sum(double v, double* red) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double t = 0.0;
  for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += red[w];
  return t;
}

// Xc[b * m + (i * d + s)] = sum_l R[i, l] A[l, s, b]     (R: dk x dk row-major)
__global__ void __launch_bounds__(256) absorb_kernel(const double* __restrict__ r, const double* __restrict__ a,
                                                     double* __restrict__ xc, int dk, int d, int dn) {
  __shared__ double sr[64][17];
  __shared__ double sa[16][65];
  const int m = dk * d;
  const int p = d * dn;            // columns of A viewed (dk, d*dn)
  const int i0 = blockIdx.y * 64, j0 = blockIdx.x * 64;
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  double acc[4][4] = {};
  for (int l0 = 0; l0 < dk; l0 += 16) {
    for (int e = threadIdx.x; e < 64 * 16; e += 256) {
      int ii = e / 16, ll = e % 16;
      sr[ii][ll] = (i0 + ii < dk && l0 + ll < dk) ? r[(int64_t)(i0 + ii) * dk + l0 + ll] : 0.0;
      int l2 = e / 64, jj = e % 64;
      sa[l2][jj] = (l0 + l2 < dk && j0 + jj < p) ? a[(int64_t)(l0 + l2) * p + j0 + jj] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int ll = 0; ll < 16; ++ll)
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[u][v] = fma(sr[ty * 4 + u][ll], sa[ll][tx * 4 + v], acc[u][v]);
    __syncthreads();
  }
  for (int u = 0; u < 4; ++u)
    for (int v = 0; v < 4; ++v) {
      int i = i0 + ty * 4 + u, j = j0 + tx * 4 + v;
      if (i < dk && j < p) {
        int s = j / dn, b = j - s * dn;
        xc[(int64_t)b * m + i * d + s] = acc[u][v];
      }
    }
  (void)m;
}

// reflector for column j of the column-major m x n matrix X (LAPACK larfg convention)
__global__ void __launch_bounds__(256) reflector_kernel(double* xc, double* tau, int m, int j) {
  __shared__ double red[4];
  double* col = xc + (int64_t)j * m;
  double s = 0.0;
  for (int i = j + 1 + threadIdx.x; i < m; i += blockDim.x) s += col[i] * col[i];
  const double sigma = block_sum(s, red);
  const double alpha = col[j];
  __syncthreads();
  if (sigma == 0.0) {
    if (threadIdx.x == 0) tau[j] = 0.0;
    return;
  }
  const double beta = -copysign(sqrt(alpha * alpha + sigma), alpha);
  const double scale = 1.0 / (alpha - beta);
  for (int i = j + 1 + threadIdx.x; i < m; i += blockDim.x) col[i] *= scale;
  if (threadIdx.x == 0) {
    tau[j] = (beta - alpha) / beta;
    col[j] = beta;
  }
}

// apply H_j = I - tau v v^T (v_j = 1, v_i = X[i, j] below) to columns c0.. of Y (m rows, column-major)
__global__ void __launch_bounds__(256) reflect_cols_kernel(const double* __restrict__ xc, const double* __restrict__ tau,
                                                           double* y, int m, int j, int c0) {
  __shared__ double red[4];
  const double t = tau[j];
  if (t == 0.0) return;
  const double* v = xc + (int64_t)j * m;
  double* col = y + (int64_t)(c0 + blockIdx.x) * m;
  double s = threadIdx.x == 0 ? col[j] : 0.0;
  for (int i = j + 1 + threadIdx.x; i < m; i += blockDim.x) s += v[i] * col[i];
  const double w = block_sum(s, red) * t;
  if (threadIdx.x == 0) col[j] -= w;
  for (int i = j + 1 + threadIdx.x; i < m; i += blockDim.x) col[i] -= w * v[i];
}

__global__ void eye_kernel(double* qc, int m, int n) {
  const int64_t total = (int64_t)m * n;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    int64_t c = e / m, i = e - c * m;
    qc[e] = (i == c) ? 1.0 : 0.0;
  }
}

// site[i, s, b] = Q[(i d + s), b] * sign(R[b, b]);  R_next[r, c] = sign(R[r, r]) * R[r, c] (upper)
__global__ void finalize_kernel(const double* __restrict__ xc, const double* __restrict__ qc, double* site,
                                double* rnext, int m, int n) {
  const int64_t total = (int64_t)m * n;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    int64_t row = e / n, b = e - row * n;   // row-major site index (row = i*d + s)
    double sg = xc[b * m + b] < 0.0 ? -1.0 : 1.0;
    site[e] = qc[b * m + row] * sg;
  }
  const int64_t tr = (int64_t)n * n;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < tr; e += (int64_t)gridDim.x * blockDim.x) {
    int64_t r = e / n, c = e - r * n;
    double sg = xc[r * m + r] < 0.0 ? -1.0 : 1.0;
    rnext[e] = (c >= r) ? sg * xc[c * m + r] : 0.0;
  }
}

__global__ void lognorm_kernel(const double* r, double* out) {
  if (threadIdx.x == 0) out[0] = log(r[0]);
}

__global__ void one_kernel(double* r) {
  if (threadIdx.x == 0) r[0] = 1.0;
}

static unsigned blocks_for(int64_t n) {
  int64_t b = (n + 255) / 256;
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>(b, 16384));
}

struct QrLayout {
  size_t x, q, r, tau, total;
};

static int32_t qr_check(int32_t n, const tn_tensor* sites, QrLayout& L) {
  if (n < 1 || !sites) return fail(TN_ERR_INVALID_ARGUMENT, "need n_sites >= 1 and sites");
  int64_t mx = 1, mr = 1;
  int64_t prev = 1;
  for (int k = 0; k < n; ++k) {
    char nm[32];
    snprintf(nm, sizeof(nm), "sites[%d]", k);
    TN_TRY(check_tensor(&sites[k], nm, TN_F64));
    const tn_tensor& t = sites[k];
    if (t.rank != 3) return fail(TN_ERR_SHAPE_MISMATCH, "%s must be rank 3", nm);
    if (t.stride[2] != 1 || t.stride[1] != t.shape[2] || t.stride[0] != t.shape[1] * t.shape[2])
      return fail(TN_ERR_UNSUPPORTED, "%s must be contiguous", nm);
    if (t.shape[0] != prev) return fail(TN_ERR_SHAPE_MISMATCH, "bond %d does not match", k);
    if (t.shape[2] > t.shape[0] * t.shape[1])
      return fail(TN_ERR_UNSUPPORTED, "%s: D_k+1 > d * D_k (wider than the row space)", nm);
    mx = std::max(mx, t.shape[0] * t.shape[1] * t.shape[2]);
    mr = std::max(mr, t.shape[2] * t.shape[2]);
    prev = t.shape[2];
  }
  if (sites[0].shape[0] != 1 || prev != 1) return fail(TN_ERR_SHAPE_MISMATCH, "boundary bonds must be 1");
  L.x = 0;
  L.q = al256(mx * 8);
  L.r = L.q + al256(mx * 8);
  L.tau = L.r + al256(std::max<int64_t>(mr, 1) * 8);
  L.total = L.tau + al256(4096 * 8);
  int64_t maxn = 1;
  for (int k = 0; k < n; ++k) maxn = std::max(maxn, sites[k].shape[2]);
  if (maxn > 4096) return fail(TN_ERR_UNSUPPORTED, "bond dimension above 4096");
  return TN_OK;
}

}  // namespace tn

using namespace tn;

extern "C" {

int32_t tn_mps_left_canonicalize_workspace(int32_t n_sites, const tn_tensor* sites, size_t* bytes) {
  if (!bytes) return fail(TN_ERR_INVALID_ARGUMENT, "bytes is NULL");
  QrLayout L;
  TN_TRY(qr_check(n_sites, sites, L));
  *bytes = L.total;
  return TN_OK;
}

int32_t tn_mps_left_canonicalize(int32_t n_sites, tn_tensor* sites, double* lognorm, void* workspace, size_t ws_bytes,
                                 void* stream) {
  QrLayout L;
  TN_TRY(qr_check(n_sites, sites, L));
  if (!lognorm) return fail(TN_ERR_INVALID_ARGUMENT, "lognorm is NULL");
  if (!workspace || ws_bytes < L.total) return fail(TN_ERR_WORKSPACE_TOO_SMALL, "workspace needs %zu bytes", L.total);
  hipStream_t st = static_cast<hipStream_t>(stream);
  char* ws = static_cast<char*>(workspace);
  double* xc = reinterpret_cast<double*>(ws + L.x);
  double* qc = reinterpret_cast<double*>(ws + L.q);
  double* r = reinterpret_cast<double*>(ws + L.r);
  double* tau = reinterpret_cast<double*>(ws + L.tau);
  hipLaunchKernelGGL(one_kernel, dim3(1), dim3(64), 0, st, r);
  for (int k = 0; k < n_sites; ++k) {
    const int dk = (int)sites[k].shape[0], d = (int)sites[k].shape[1], dn = (int)sites[k].shape[2];
    const int m = dk * d, n = dn;
    double* a = static_cast<double*>(sites[k].data);
    dim3 g((unsigned)((d * dn + 63) / 64), (unsigned)((dk + 63) / 64));
    hipLaunchKernelGGL(absorb_kernel, g, dim3(256), 0, st, r, a, xc, dk, d, dn);
    for (int j = 0; j < n; ++j) {
      hipLaunchKernelGGL(reflector_kernel, dim3(1), dim3(256), 0, st, xc, tau, m, j);
      if (j + 1 < n) hipLaunchKernelGGL(reflect_cols_kernel, dim3(n - j - 1), dim3(256), 0, st, xc, tau, xc, m, j, j + 1);
    }
    hipLaunchKernelGGL(eye_kernel, dim3(blocks_for((int64_t)m * n)), dim3(256), 0, st, qc, m, n);
    for (int j = n - 1; j >= 0; --j)
      hipLaunchKernelGGL(reflect_cols_kernel, dim3(n - j), dim3(256), 0, st, xc, tau, qc, m, j, j);
    hipLaunchKernelGGL(finalize_kernel, dim3(blocks_for((int64_t)m * n)), dim3(256), 0, st, xc, qc, a, r, m, n);
    TN_TRY(hip_check(hipGetLastError(), "canonicalize"));
  }
  hipLaunchKernelGGL(lognorm_kernel, dim3(1), dim3(64), 0, st, r, lognorm);
  return hip_check(hipGetLastError(), "lognorm");
}

}  // extern "C"
