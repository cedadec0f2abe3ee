// Left-canonical gauge of an MPS in FP64 on the GPU: successive Householder
// QR factorisations (Golub and Van Loan, "Matrix Computations", 5.1-5.2).
// For site k the carried triangular factor is absorbed first
// (X = R_{k-1} A_k viewed as (D_k d) x D_{k+1}), X is factorised in place,
// the thin Q is accumulated backwards from [I; 0], and signs are fixed so
// that diag(R) >= 0.  X and Q are kept column-major so every reflector and
// column update reads contiguous memory.
// Up to 2048 rows the factorisation is blocked in the compact WY form
// (Schreiber and Van Loan; Golub and Van Loan 5.2.3): a panel of 16 columns
// is factorised by one workgroup holding the panel in registers (two
// workgroup reductions per column, row conditions as selects so the unrolled
// panel stays short), which then forms the panel's triangular factor T from
// the Gram matrix of its reflectors; one launch applies
// I - V T^T V^T to all trailing columns (one reduction per workgroup); Q is
// accumulated panel by panel in reverse with I - V T V^T.
// Taller matrices take one reflector launch and one update launch per column.
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

// Xc[b * m + (i * d + s)] = sum_l R[i, l] A[l, s, b]     (R: dk x dk row-major,
// upper triangular: the sum starts at l = i, so a row block skips the l
// blocks below it).  The 64 x 64 result tile goes through LDS so that the
// column-major stores run along i.
__global__ void __launch_bounds__(256) absorb_kernel(const double* __restrict__ r, const double* __restrict__ a,
                                                     double* __restrict__ xc, int dk, int d, int dn) {
  __shared__ double sr[64][17];
  __shared__ double sa[16][65];
  __shared__ double so[64][65];
  const int m = dk * d;
  const int p = d * dn;            // columns of A viewed (dk, d*dn)
  const int i0 = blockIdx.y * 64, j0 = blockIdx.x * 64;
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  double acc[4][4] = {};
  for (int l0 = i0; l0 < dk; l0 += 16) {
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
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) so[ty * 4 + u][tx * 4 + v] = acc[u][v];
  __syncthreads();
  // consecutive threads take consecutive i of one column j = (s, b)
  for (int e = threadIdx.x; e < 64 * 64; e += 256) {
    const int jl = e / 64, il = e % 64;
    const int i = i0 + il, j = j0 + jl;
    if (i < dk && j < p) {
      const int s = j / dn, b = j - s * dn;
      xc[(int64_t)b * m + i * d + s] = so[il][jl];
    }
  }
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

// ---- blocked path (m <= kQrThreads * kQrRows) --------------------------------

constexpr int kQrThreads = 512;   // threads per workgroup; thread t owns rows t + 512 q
constexpr int kQrRows = 4;        // rows per thread
constexpr int kQrNb = 16;         // panel width
constexpr int kQrCb = 4;          // trailing columns per workgroup
constexpr int kQrWaves = kQrThreads / 64;

// x from lane (this lane xor M) of the wavefront.  Within a 16-lane row (M <
// 16) a DPP move on each 32-bit half: quad permutations for M = 1, 2, the
// row rotation by 8 for M = 8, and for M = 4 the rotation by 4 or by 12 as
// the lane's bit 2 is set or clear; across rows a lane exchange through the
// LDS crossbar.
template <int CTRL>
__device__ __forceinline__ double qr_dpp(double x) {
  const long long v = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)v, CTRL, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(v >> 32), CTRL, 0xf, 0xf, false);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned int)lo);
}

template <int M>
__device__ __forceinline__ double qr_xor_lane(double x) {
  if constexpr (M == 1) return qr_dpp<0xB1>(x);         // quad_perm [1, 0, 3, 2]
  else if constexpr (M == 2) return qr_dpp<0x4E>(x);    // quad_perm [2, 3, 0, 1]
  else if constexpr (M == 4) {
    // row_ror n: lane i reads lane (i - n) mod 16 of its row
    const double below = qr_dpp<0x124>(x);              // row_ror 4: lane i - 4
    const double above = qr_dpp<0x12C>(x);              // row_ror 12: lane i + 4
    return (threadIdx.x & 4) ? below : above;
  } else if constexpr (M == 8) return qr_dpp<0x128>(x);  // row_ror 8: lane i xor 8
  else return __shfl_xor(x, M, 64);
}

// x of lane L (a constant) in every lane
template <int L>
__device__ __forceinline__ double qr_read_lane(double x) {
  const long long v = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_readlane((int)v, L);
  const int hi = __builtin_amdgcn_readlane((int)(v >> 32), L);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned int)lo);
}

template <int NV, int I = 0>
__device__ __forceinline__ void qr_broadcast(double t, double (&v)[NV]) {
  if constexpr (I < NV) {
    v[I] = qr_read_lane<I>(t);
    qr_broadcast<NV, I + 1>(t, v);
  }
}

// Wavefront reduce-scatter of N partial values (N a power of two <= 64):
// lane l returns the sum over the 64 lanes of value l % N.  Each halving step
// sends one half of the remaining values to the partner lane and keeps the
// other half (N - 1 exchanges in all, instead of 6 N for N separate sums).
template <int N, int H>
__device__ __forceinline__ void qr_halve(double (&v)[N], int lane) {
  if constexpr (H >= 1) {
    const bool up = (lane & H) != 0;
#pragma unroll
    for (int i = 0; i < H; ++i) {
      const double send = up ? v[i] : v[i + H];
      const double keep = up ? v[i + H] : v[i];
      v[i] = keep + qr_xor_lane<H>(send);
    }
    qr_halve<N, H / 2>(v, lane);
  }
}

// r summed over the lane groups that differ in bits N, 2N, ... 32
template <int MK>
__device__ __forceinline__ void qr_xor_tail(double& r) {
  if constexpr (MK < 64) {
    r += qr_xor_lane<MK>(r);
    qr_xor_tail<MK * 2>(r);
  }
}

template <int N>
__device__ inline double qr_reduce_scatter(double (&v)[N]) {
  const int lane = threadIdx.x & 63;
  qr_halve<N, N / 2>(v, lane);
  double r = v[0];
  qr_xor_tail<N>(r);
  return r;
}

// Workgroup sum of v[0..NV) returned to every thread.  P (a power of two >=
// NV) values per wavefront go through red[buf] (two buffers used in turn, so
// one barrier per reduction suffices: a wavefront can only write a buffer
// again after every wavefront has passed the barrier of the reduction that
// read it last).
template <int NV, int P>
__device__ inline void qr_block_sum(double (&v)[NV], double (*red)[kQrWaves * 64], int& buf) {
  double w[P];
#pragma unroll
  for (int i = 0; i < P; ++i) w[i] = i < NV ? v[i] : 0.0;
  const double r = qr_reduce_scatter<P>(w);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane < P) red[buf][wave * P + lane] = r;
  __syncthreads();
  // lane i < NV of every wavefront adds the wavefronts' partial sums of value
  // i (in wavefront order), and every lane takes value i from lane i: eight
  // LDS reads per lane instead of eight per value
  double t = 0.0;
  if (lane < NV) {
#pragma unroll
    for (int wv = 0; wv < kQrWaves; ++wv) t += red[buf][wv * P + lane];
  }
  qr_broadcast<NV>(t, v);
  buf ^= 1;
}

// the reflector of panel column J (a template argument, so the register
// panel is only indexed by constants), then its update of the panel columns
// to its right; the same arithmetic as reflector_kernel + reflect_cols_kernel.
// Row conditions are selects, not branches, to keep the unrolled panel short.
template <int J>
__device__ __forceinline__ void qr_panel_step(double (&x)[kQrRows][kQrNb], double (*red)[kQrWaves * 64], int& buf,
                                              double* tau, int m, int j0, int nb) {
  if constexpr (J < kQrNb) {
    if (J < nb) {
      const int gj = j0 + J;
      double s[2] = {0.0, 0.0};   // sigma (rows below gj), alpha (row gj)
#pragma unroll
      for (int q = 0; q < kQrRows; ++q) {
        const int row = threadIdx.x + kQrThreads * q;
        const double xv = x[q][J];
        s[0] += (row > gj && row < m) ? xv * xv : 0.0;
        s[1] += row == gj ? xv : 0.0;
      }
      qr_block_sum<2, 2>(s, red, buf);
      const double sigma = s[0], alpha = s[1];
      double t = 0.0;
      if (sigma != 0.0) {
        const double beta = -copysign(sqrt(alpha * alpha + sigma), alpha);
        const double scale = 1.0 / (alpha - beta);
        t = (beta - alpha) / beta;
#pragma unroll
        for (int q = 0; q < kQrRows; ++q) {
          const int row = threadIdx.x + kQrThreads * q;
          const double xv = x[q][J];
          x[q][J] = (row > gj && row < m) ? xv * scale : (row == gj ? beta : xv);
        }
      }
      if (threadIdx.x == 0) tau[gj] = t;
      if constexpr (J + 1 < kQrNb) {
        // t is the same in every thread, so the barriers inside are reached by all
        if (t != 0.0 && J + 1 < nb) {
          constexpr int NW = kQrNb - J - 1;
          double v[kQrRows];   // the reflector at this thread's rows: 1 at gj, X below, 0 above
#pragma unroll
          for (int q = 0; q < kQrRows; ++q) {
            const int row = threadIdx.x + kQrThreads * q;
            v[q] = (row > gj && row < m) ? x[q][J] : (row == gj ? 1.0 : 0.0);
          }
          double w[NW];
#pragma unroll
          for (int c = 0; c < NW; ++c) {
            w[c] = 0.0;
#pragma unroll
            for (int q = 0; q < kQrRows; ++q) w[c] += v[q] * x[q][J + 1 + c];
          }
          qr_block_sum<NW, (NW > 8 ? 16 : NW > 4 ? 8 : NW > 2 ? 4 : NW > 1 ? 2 : 1)>(w, red, buf);
#pragma unroll
          for (int c = 0; c < NW; ++c) {
            const double tw = t * w[c];
#pragma unroll
            for (int q = 0; q < kQrRows; ++q) x[q][J + 1 + c] -= tw * v[q];
          }
        }
      }
    }
    qr_panel_step<J + 1>(x, red, buf, tau, m, j0, nb);
  }
}

// Factorise columns j0 .. j0+nb-1 (rows j0..m-1) of the column-major X in
// place, then form the panel's triangular factor (LAPACK larft, forward,
// columnwise): H_0 ... H_{nb-1} = I - V T V^T with T[j][j] = tau_j and
// T[0:j, j] = -tau_j T[0:j, 0:j] (V[:, 0:j]^T v_j); T row-major 16 x 16.
__global__ void __launch_bounds__(kQrThreads) qr_panel_kernel(double* xc, double* tau, double* tf, int m, int j0,
                                                              int nb) {
  __shared__ double red[2][kQrWaves * 64];
  __shared__ double gram[kQrNb * kQrNb];
  __shared__ double tl[kQrNb * kQrNb];
  int buf = 0;
  double x[kQrRows][kQrNb];
#pragma unroll
  for (int q = 0; q < kQrRows; ++q) {
    const int row = threadIdx.x + kQrThreads * q;
#pragma unroll
    for (int c = 0; c < kQrNb; ++c) x[q][c] = (row < m && c < nb) ? xc[(int64_t)(j0 + c) * m + row] : 0.0;
  }
  qr_panel_step<0>(x, red, buf, tau, m, j0, nb);
#pragma unroll
  for (int q = 0; q < kQrRows; ++q) {
    const int row = threadIdx.x + kQrThreads * q;
    if (row < m) {
#pragma unroll
      for (int c = 0; c < kQrNb; ++c)
        if (c < nb) xc[(int64_t)(j0 + c) * m + row] = x[q][c];
    }
  }
  // the reflectors in place of the panel: v_c is 1 at row j0 + c, X below it,
  // 0 above (and 0 in the columns past nb)
#pragma unroll
  for (int q = 0; q < kQrRows; ++q) {
    const int row = threadIdx.x + kQrThreads * q;
#pragma unroll
    for (int c = 0; c < kQrNb; ++c) {
      const int gc = j0 + c;
      x[q][c] = (c >= nb || row >= m) ? 0.0 : (row == gc ? 1.0 : (row > gc ? x[q][c] : 0.0));
    }
  }
  // Gram entries v_i . v_j (i < j), enumerated column by column: 120 pairs in
  // batches of 16 (registers: the panel holds 128)
  constexpr int kPairs = kQrNb * (kQrNb - 1) / 2;
#pragma unroll
  for (int b0 = 0; b0 < kPairs; b0 += 16) {
    double g[16];
#pragma unroll
    for (int p = 0; p < 16; ++p) {
      g[p] = 0.0;
      const int pp = b0 + p;
      if (pp < kPairs) {
        int j = 1, base = 0;
#pragma unroll
        for (int jj = 1; jj < kQrNb; ++jj)
          if (pp >= jj * (jj - 1) / 2) {
            j = jj;
            base = jj * (jj - 1) / 2;
          }
        const int i = pp - base;
#pragma unroll
        for (int q = 0; q < kQrRows; ++q) g[p] += x[q][i] * x[q][j];
      }
    }
    const double v = qr_reduce_scatter<16>(g);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane < 16) red[buf][wave * 16 + lane] = v;
    __syncthreads();
    if (threadIdx.x < 16 && b0 + (int)threadIdx.x < kPairs) {
      double t = 0.0;
#pragma unroll
      for (int wv = 0; wv < kQrWaves; ++wv) t += red[buf][wv * 16 + threadIdx.x];
      gram[b0 + threadIdx.x] = t;   // packed pair order
    }
    buf ^= 1;
  }
  __syncthreads();
  // lane i builds row i of T: T[i][j] needs only T[i][i..j-1] (its own row)
  if (threadIdx.x < kQrNb) {
    const int i = threadIdx.x;
    double row[kQrNb];
#pragma unroll
    for (int j = 0; j < kQrNb; ++j) {
      const double tj = j < nb ? tau[j0 + j] : 0.0;
      double v = 0.0;
      if (i < j) {
#pragma unroll
        for (int l = 0; l < j; ++l)
          if (l >= i) v += row[l] * gram[j * (j - 1) / 2 + l];
        v *= -tj;
      } else if (i == j) {
        v = tj;
      }
      row[j] = v;
    }
#pragma unroll
    for (int j = 0; j < kQrNb; ++j) tl[i * kQrNb + j] = row[j];
  }
  __syncthreads();
  for (int e = threadIdx.x; e < kQrNb * kQrNb; e += kQrThreads) tf[(j0 / kQrNb) * kQrNb * kQrNb + e] = tl[e];
}

// reflector j of the panel at this thread's rows: 1 at row j0+j, X below, 0 above
__device__ inline void qr_load_v(const double* __restrict__ xc, int m, int j0, int nb, int j, double (&v)[kQrRows]) {
  const int gj = j0 + j;
#pragma unroll
  for (int q = 0; q < kQrRows; ++q) {
    const int row = threadIdx.x + kQrThreads * q;
    v[q] = j >= nb ? 0.0 : (row == gj ? 1.0 : ((row > gj && row < m) ? xc[(int64_t)gj * m + row] : 0.0));
  }
}

// apply the panel j0 .. j0+nb-1 (reflectors in X, triangular factor T) to
// columns c0 .. c0+ncols-1 of Y: Y -= V T^T (V^T Y) in the factorisation
// (transpose = 1: H_{nb-1} ... H_0 Y), Y -= V T (V^T Y) for the accumulation
// of Q (transpose = 0: H_0 ... H_{nb-1} Y)
__global__ void __launch_bounds__(kQrThreads) qr_apply_kernel(const double* __restrict__ xc,
                                                              const double* __restrict__ tf, double* y, int m, int j0,
                                                              int nb, int c0, int ncols, int transpose) {
  constexpr int NW = kQrNb * kQrCb;   // 64 entries of W = V^T Y
  __shared__ double red[kQrWaves * NW];
  __shared__ double sw[NW], sw2[NW], st[kQrNb * kQrNb];
  for (int e = threadIdx.x; e < kQrNb * kQrNb; e += kQrThreads) st[e] = tf[(j0 / kQrNb) * kQrNb * kQrNb + e];
  const int cb0 = c0 + blockIdx.x * kQrCb;
  double yv[kQrRows][kQrCb];
#pragma unroll
  for (int q = 0; q < kQrRows; ++q) {
    const int row = threadIdx.x + kQrThreads * q;
#pragma unroll
    for (int c = 0; c < kQrCb; ++c)
      yv[q][c] = (row < m && cb0 + c < c0 + ncols) ? y[(int64_t)(cb0 + c) * m + row] : 0.0;
  }
  double w[NW];
#pragma unroll
  for (int j = 0; j < kQrNb; ++j) {
    double v[kQrRows];
    qr_load_v(xc, m, j0, nb, j, v);
#pragma unroll
    for (int c = 0; c < kQrCb; ++c) {
      double s = 0.0;
#pragma unroll
      for (int q = 0; q < kQrRows; ++q) s += v[q] * yv[q][c];
      w[j * kQrCb + c] = s;
    }
  }
  const double r = qr_reduce_scatter<NW>(w);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  red[wave * NW + lane] = r;
  __syncthreads();
  if (threadIdx.x < NW) {
    double t = 0.0;
#pragma unroll
    for (int wv = 0; wv < kQrWaves; ++wv) t += red[wv * NW + threadIdx.x];
    sw[threadIdx.x] = t;
  }
  __syncthreads();
  if (threadIdx.x < NW) {
    const int j = threadIdx.x / kQrCb, c = threadIdx.x % kQrCb;
    double t = 0.0;
#pragma unroll
    for (int l = 0; l < kQrNb; ++l) t += (transpose ? st[l * kQrNb + j] : st[j * kQrNb + l]) * sw[l * kQrCb + c];
    sw2[threadIdx.x] = t;
  }
  __syncthreads();
#pragma unroll 2
  for (int j = 0; j < kQrNb; ++j) {
    double v[kQrRows];
    qr_load_v(xc, m, j0, nb, j, v);
#pragma unroll
    for (int c = 0; c < kQrCb; ++c) {
      const double w2 = sw2[j * kQrCb + c];
#pragma unroll
      for (int q = 0; q < kQrRows; ++q) yv[q][c] -= v[q] * w2;
    }
  }
#pragma unroll
  for (int q = 0; q < kQrRows; ++q) {
    const int row = threadIdx.x + kQrThreads * q;
    if (row < m) {
#pragma unroll
      for (int c = 0; c < kQrCb; ++c)
        if (cb0 + c < c0 + ncols) y[(int64_t)(cb0 + c) * m + row] = yv[q][c];
    }
  }
}

__global__ void eye_kernel(double* qc, int m, int n) {
  const int64_t total = (int64_t)m * n;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    int64_t c = e / m, i = e - c * m;
    qc[e] = (i == c) ? 1.0 : 0.0;
  }
}

// site[i, s, b] = Q[(i d + s), b] * sign(R[b, b]);  R_next[r, c] = sign(R[r, r]) * R[r, c] (upper)
// Q with column signs so that diag(R) >= 0, written over the site
__global__ void finalize_q_kernel(const double* __restrict__ xc, const double* __restrict__ qc, double* site, int m,
                                  int n) {
  const int64_t total = (int64_t)m * n;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    int64_t row = e / n, b = e - row * n;   // row-major site index (row = i*d + s)
    double sg = xc[b * m + b] < 0.0 ? -1.0 : 1.0;
    site[e] = qc[b * m + row] * sg;
  }
}

// R with row signs (diag(R) >= 0), row-major, for the next site's absorb
__global__ void finalize_r_kernel(const double* __restrict__ xc, double* rnext, int m, int n) {
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

// X, Q and T come in two sets, used by alternate sites: a site's Q is formed
// on the side stream while the next site is factorised
// Householder QR of a column-major m x n matrix (m >= n) for other callers:
// the blocked path only (m <= 2048), factorised in place (R in the upper
// triangle, the reflectors below), T factors in tf; and the product Q y.
bool householder_qr_fits(int64_t m) { return m <= (int64_t)kQrThreads * kQrRows; }

size_t householder_tf_doubles(int64_t n) { return (size_t)((n + kQrNb - 1) / kQrNb) * kQrNb * kQrNb; }

int32_t householder_qr(double* xc, int m, int n, double* tau, double* tf, hipStream_t st) {
  for (int j0 = 0; j0 < n; j0 += kQrNb) {
    const int nb = std::min(kQrNb, n - j0);
    hipLaunchKernelGGL(qr_panel_kernel, dim3(1), dim3(kQrThreads), 0, st, xc, tau, tf, m, j0, nb);
    const int rest = n - j0 - nb;
    if (rest > 0)
      hipLaunchKernelGGL(qr_apply_kernel, dim3((unsigned)((rest + kQrCb - 1) / kQrCb)), dim3(kQrThreads), 0, st, xc, tf,
                         xc, m, j0, nb, j0 + nb, rest, 1);
  }
  return hip_check(hipGetLastError(), "householder qr");
}

// y (m x ncols, column-major) := Q y, the panels applied last to first
int32_t householder_apply_q(const double* xc, int m, int n, const double* tf, double* y, int ncols, hipStream_t st) {
  for (int j0 = (n - 1) / kQrNb * kQrNb; j0 >= 0; j0 -= kQrNb) {
    const int nb = std::min(kQrNb, n - j0);
    hipLaunchKernelGGL(qr_apply_kernel, dim3((unsigned)((ncols + kQrCb - 1) / kQrCb)), dim3(kQrThreads), 0, st, xc, tf,
                       y, m, j0, nb, 0, ncols, 0);
  }
  return hip_check(hipGetLastError(), "householder apply");
}

struct QrLayout {
  size_t x[2], q[2], r, tau, tf[2], total;
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
  size_t o = 0;
  for (int h = 0; h < 2; ++h) {
    L.x[h] = o;
    o += al256(mx * 8);
    L.q[h] = o;
    o += al256(mx * 8);
    L.tf[h] = o;
    o += al256((4096 / kQrNb) * kQrNb * kQrNb * 8);
  }
  L.r = o;
  o += al256(std::max<int64_t>(mr, 1) * 8);
  L.tau = o;
  o += al256(4096 * 8);
  L.total = o;
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
  double* r = reinterpret_cast<double*>(ws + L.r);
  double* tau = reinterpret_cast<double*>(ws + L.tau);
  // Site k's factorisation and R run on the caller's stream; its Q (the
  // reflectors applied to [I; 0]) and the write-back run on the side stream,
  // overlapping site k+1's factorisation, whose one-workgroup panels leave
  // most of the chip idle.  Site k+2 reuses site k's X, Q and T only after
  // that Q is done (event per set); the call ends joined on the caller's stream.
  hipStream_t side = st;
  TN_TRY(side_stream(side));
  hipEvent_t ev_fact = nullptr, ev_q[2] = {nullptr, nullptr};
  struct EventGuard {
    hipEvent_t* e[3];
    ~EventGuard() {
      for (hipEvent_t* p : e)
        if (*p) hipEventDestroy(*p);
    }
  } guard{{&ev_fact, &ev_q[0], &ev_q[1]}};
  for (hipEvent_t* e : guard.e)
    if (hipEventCreateWithFlags(e, hipEventDisableTiming) != hipSuccess) return fail(TN_ERR_DEVICE, "create event failed");
  hipEventRecord(ev_q[0], st);
  hipEventRecord(ev_q[1], st);
  hipLaunchKernelGGL(one_kernel, dim3(1), dim3(64), 0, st, r);
  int32_t rc = TN_OK;
  for (int k = 0; k < n_sites && rc == TN_OK; ++k) {
    const int h = k & 1;
    double* xc = reinterpret_cast<double*>(ws + L.x[h]);
    double* qc = reinterpret_cast<double*>(ws + L.q[h]);
    double* tf = reinterpret_cast<double*>(ws + L.tf[h]);
    const int dk = (int)sites[k].shape[0], d = (int)sites[k].shape[1], dn = (int)sites[k].shape[2];
    const int m = dk * d, n = dn;
    double* a = static_cast<double*>(sites[k].data);
    hipStreamWaitEvent(st, ev_q[h], 0);   // site k-2's Q no longer reads this set
    dim3 g((unsigned)((d * dn + 63) / 64), (unsigned)((dk + 63) / 64));
    hipLaunchKernelGGL(absorb_kernel, g, dim3(256), 0, st, r, a, xc, dk, d, dn);
    const bool blocked = m <= kQrThreads * kQrRows;
    if (blocked) {
      for (int j0 = 0; j0 < n; j0 += kQrNb) {
        const int nb = std::min(kQrNb, n - j0);
        hipLaunchKernelGGL(qr_panel_kernel, dim3(1), dim3(kQrThreads), 0, st, xc, tau, tf, m, j0, nb);
        const int rest = n - j0 - nb;
        if (rest > 0)
          hipLaunchKernelGGL(qr_apply_kernel, dim3((unsigned)((rest + kQrCb - 1) / kQrCb)), dim3(kQrThreads), 0, st, xc,
                             tf, xc, m, j0, nb, j0 + nb, rest, 1);
      }
    } else {
      for (int j = 0; j < n; ++j) {
        hipLaunchKernelGGL(reflector_kernel, dim3(1), dim3(256), 0, st, xc, tau, m, j);
        if (j + 1 < n) hipLaunchKernelGGL(reflect_cols_kernel, dim3(n - j - 1), dim3(256), 0, st, xc, tau, xc, m, j, j + 1);
      }
    }
    hipLaunchKernelGGL(finalize_r_kernel, dim3(blocks_for((int64_t)n * n)), dim3(256), 0, st, xc, r, m, n);
    // Q: on the side stream for the blocked path; the column path's Q needs
    // tau, which the next site overwrites, so it stays on the caller's stream
    hipStream_t qs = blocked ? side : st;
    if (blocked) {
      hipEventRecord(ev_fact, st);
      hipStreamWaitEvent(side, ev_fact, 0);
    }
    hipLaunchKernelGGL(eye_kernel, dim3(blocks_for((int64_t)m * n)), dim3(256), 0, qs, qc, m, n);
    if (blocked) {
      for (int j0 = (n - 1) / kQrNb * kQrNb; j0 >= 0; j0 -= kQrNb) {
        const int nb = std::min(kQrNb, n - j0);
        hipLaunchKernelGGL(qr_apply_kernel, dim3((unsigned)((n - j0 + kQrCb - 1) / kQrCb)), dim3(kQrThreads), 0, qs, xc,
                           tf, qc, m, j0, nb, j0, n - j0, 0);
      }
    } else {
      for (int j = n - 1; j >= 0; --j)
        hipLaunchKernelGGL(reflect_cols_kernel, dim3(n - j), dim3(256), 0, qs, xc, tau, qc, m, j, j);
    }
    hipLaunchKernelGGL(finalize_q_kernel, dim3(blocks_for((int64_t)m * n)), dim3(256), 0, qs, xc, qc, a, m, n);
    hipEventRecord(ev_q[h], qs);
    rc = hip_check(hipGetLastError(), "canonicalize");
  }
  // join: every Q written back before the call's later work on the caller's stream
  hipStreamWaitEvent(st, ev_q[0], 0);
  hipStreamWaitEvent(st, ev_q[1], 0);
  TN_TRY(rc);
  hipLaunchKernelGGL(lognorm_kernel, dim3(1), dim3(64), 0, st, r, lognorm);
  return hip_check(hipGetLastError(), "lognorm");
}

}  // extern "C"
