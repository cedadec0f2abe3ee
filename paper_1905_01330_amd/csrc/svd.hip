// Node splitting (section III.B "Node Splitting"; Appendix A "Saving
// Memory") by an FP64 singular value decomposition on the GPU.
//
// The node is read as the matrix A[(left legs), (right legs)] and copied into
// a column-major FP64 work matrix W whose rows are the longer side (R) and
// whose columns the shorter (C), so W = A or W = A^T.  One-sided Jacobi
// (Hestenes) makes the columns of W mutually orthogonal by plane rotations
// applied from the right, accumulated in V (W_final = W_0 V): then the
// column norms are the singular values, the normalised columns one set of
// singular vectors and V the other.
//
// Blocked form: the columns are cut into blocks of KB; in each round of a
// sweep the blocks are paired by the circle method (every pair of blocks
// meets once per sweep) and one workgroup per pair
//   1. loads the pair's 2KB columns X into LDS,
//   2. runs cyclic one-sided Jacobi on them, KB disjoint column pairs at a
//      time, each rotation computed from the dot products of the current
//      columns (the 2x2 symmetric Schur step, Golub and Van Loan, "Matrix
//      Computations", section 8.5, on [a.a a.b; a.b b.b]), accumulating the
//      rotations in J,
//   3. writes X back and replaces the same columns of V by V J.
// Rotations taken from the current columns, not from an updated Gram
// matrix, keep the small singular values accurate when a pair mixes large
// and tiny columns.  KB is the one of 8, 4, 2, 1 with the cheapest modelled
// sweep among those whose block pair fits in LDS for the number of rows;
// when none fits (about 9600 rows) the pair kernel forms the Gram matrix
// instead and diagonalises it in LDS (accurate to eps times the largest
// singular value only).
// Before every sweep the columns are ranked by norm and the blocks take them
// in that order (a permutation table, no data moves): pairing columns of
// similar size first cuts the sweeps needed on graded spectra by a third.
// A pair whose columns are already orthogonal to the tolerance is left
// alone; the host ends the sweeps when a sweep rotated no pair.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "internal.h"

namespace tn {

namespace {

constexpr int kB = 16;          // columns per block
constexpr int kP = 2 * kB;      // columns of a block pair (order of the Gram matrix)
constexpr int kNT = 256;        // threads of the pair kernel
constexpr int kRows = 64;       // rows staged per chunk
constexpr int kMaxSweeps = 100;
constexpr int kPrecondMinCols = 32;   // narrower nodes converge in a few sweeps anyway
constexpr int kInnerSweeps = 14;

// Strided matrix view of the node: element (i, j) at p + off(i over rows) + off(j over cols)
struct MatView {
  const void* p;
  int32_t dtype;
  int32_t nr, nc;                 // axes of the row / column multi-index
  int64_t rdim[TN_MAX_RANK], rst[TN_MAX_RANK];
  int64_t cdim[TN_MAX_RANK], cst[TN_MAX_RANK];
};

__device__ inline int64_t multi_off(int64_t idx, int n, const int64_t* dim, const int64_t* st) {
  int64_t o = 0;
  for (int a = n - 1; a >= 0; --a) {
    const int64_t q = idx / dim[a];
    o += (idx - q * dim[a]) * st[a];
    idx = q;
  }
  return o;
}

// W[r + R * c] = A(i, j) with (r, c) = (i, j) or (j, i); columns c >= C (the
// padding up to whole blocks) are zero.  V = identity (Cp x Cp).
__global__ void svd_gather_kernel(MatView a, int transposed, int64_t R, int64_t C, int64_t Cp, double* W, double* V) {
  const int64_t nw = R * Cp, nv = Cp * Cp;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nw + nv; e += (int64_t)gridDim.x * blockDim.x) {
    if (e < nw) {
      const int64_t r = e % R, c = e / R;
      double x = 0.0;
      if (c < C) {
        const int64_t i = transposed ? c : r, j = transposed ? r : c;
        const int64_t off = multi_off(i, a.nr, a.rdim, a.rst) + multi_off(j, a.nc, a.cdim, a.cst);
        x = a.dtype == TN_F64 ? static_cast<const double*>(a.p)[off] : (double)static_cast<const float*>(a.p)[off];
      }
      W[e] = x;
    } else {
      const int64_t f = e - nw;
      V[f] = (f % Cp) == (f / Cp) ? 1.0 : 0.0;
    }
  }
}

// block pair `pair` of round `round` (nb blocks, nb even): the circle method
// keeps block nb-1 fixed and rotates the others
__device__ inline void round_pair(int nb, int round, int pair, int& p, int& q) {
  const int m = nb - 1;
  if (pair == 0) {
    p = m;
    q = round % m;
  } else {
    p = (round + pair) % m;
    q = (round - pair + m) % m;
  }
}

// the same schedule for kP indices inside the pair kernel
__device__ inline void inner_pair(int step, int i, int& a, int& b) {
  constexpr int m = kP - 1;
  if (i == 0) {
    a = m;
    b = step;
  } else {
    a = (step + i) % m;
    b = (step - i + m) % m;
  }
}

struct PairSmem {
  double G[kP][kP + 1];
  double J[kP][kP + 1];
  double X[kRows][kP + 1];
  double cs[kB][2];
  int ab[kB][2];
  double red;
  int flag;
};

// X <- X J for rows [0, nrows) of the kP columns col[0..kP) of M (leading dimension ld)
__device__ void apply_rotation(double* M, int64_t ld, int64_t nrows, const int* col, PairSmem& sm) {
  const int tid = threadIdx.x;
  for (int64_t r0 = 0; r0 < nrows; r0 += kRows) {
    const int nr = nrows - r0 < kRows ? (int)(nrows - r0) : kRows;
    for (int e = tid; e < kRows * kP; e += kNT) {
      const int c = e / kRows, r = e % kRows;
      sm.X[r][c] = r < nr ? M[(int64_t)col[c] * ld + r0 + r] : 0.0;
    }
    __syncthreads();
    for (int e = tid; e < kRows * kP; e += kNT) {
      const int c = e / kRows, r = e % kRows;
      if (r < nr) {
        double s = 0.0;
#pragma unroll 8
        for (int i = 0; i < kP; ++i) s += sm.X[r][i] * sm.J[i][c];
        M[(int64_t)col[c] * ld + r0 + r] = s;
      }
    }
    __syncthreads();
  }
}

__global__ void __launch_bounds__(kNT) jacobi_pair_kernel(double* W, double* V, int64_t R, int64_t Cp, int nb,
                                                         int round, double tol, int* rotated, const int* perm) {
  __shared__ PairSmem sm;
  const int tid = threadIdx.x;
  int p, q;
  round_pair(nb, round, blockIdx.x, p, q);
  int col[kP];
#pragma unroll
  for (int c = 0; c < kP; ++c) col[c] = perm[c < kB ? p * kB + c : q * kB + (c - kB)];

  // 1. Gram matrix of the pair's columns, rows staged through LDS
  double g[4] = {0.0, 0.0, 0.0, 0.0};
  for (int64_t r0 = 0; r0 < R; r0 += kRows) {
    const int nr = R - r0 < kRows ? (int)(R - r0) : kRows;
    for (int e = tid; e < kRows * kP; e += kNT) {
      const int c = e / kRows, r = e % kRows;
      sm.X[r][c] = r < nr ? W[(int64_t)col[c] * R + r0 + r] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int e = tid + t * kNT, i = e / kP, j = e % kP;
      double s = 0.0;
      for (int r = 0; r < nr; ++r) s += sm.X[r][i] * sm.X[r][j];
      g[t] += s;
    }
    __syncthreads();
  }
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int e = tid + t * kNT, i = e / kP, j = e % kP;
    sm.G[i][j] = g[t];
    sm.J[i][j] = i == j ? 1.0 : 0.0;
  }
  if (tid == 0) sm.flag = 0;
  __syncthreads();

  // the pair needs work when two of its columns are not orthogonal to the tolerance
  auto off_exceeds = [&](double lim) {
    bool any = false;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int e = tid + t * kNT, i = e / kP, j = e % kP;
      if (i < j) {
        const double d = sm.G[i][i] * sm.G[j][j];
        if (d > 0.0 && fabs(sm.G[i][j]) > lim * sqrt(d)) any = true;
      }
    }
    return any;
  };
  if (off_exceeds(tol)) sm.flag = 1;
  __syncthreads();
  if (!sm.flag) return;
  if (tid == 0) atomicAdd(rotated, 1);

  // 2. cyclic Jacobi on G: kB disjoint rotations per step, kP - 1 steps per sweep
  for (int sweep = 0; sweep < kInnerSweeps; ++sweep) {
    for (int step = 0; step < kP - 1; ++step) {
      if (tid < kB) {
        int a, b;
        inner_pair(step, tid, a, b);
        if (a > b) {
          const int t = a;
          a = b;
          b = t;
        }
        const double app = sm.G[a][a], aqq = sm.G[b][b], apq = sm.G[a][b];
        double c = 1.0, s = 0.0;
        if (apq != 0.0 && fabs(apq) > 1e-300) {
          const double tau = (aqq - app) / (2.0 * apq);
          const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
          c = 1.0 / sqrt(1.0 + t * t);
          s = t * c;
        }
        sm.cs[tid][0] = c;
        sm.cs[tid][1] = s;
        sm.ab[tid][0] = a;
        sm.ab[tid][1] = b;
      }
      __syncthreads();
      // rows a, b of G <- J^T G
      for (int e = tid; e < kB * kP; e += kNT) {
        const int pi = e / kP, x = e % kP;
        const int a = sm.ab[pi][0], b = sm.ab[pi][1];
        const double c = sm.cs[pi][0], s = sm.cs[pi][1];
        const double ga = sm.G[a][x], gb = sm.G[b][x];
        sm.G[a][x] = c * ga - s * gb;
        sm.G[b][x] = s * ga + c * gb;
      }
      __syncthreads();
      // columns a, b of G <- G J, and of J <- J J_step
      for (int e = tid; e < kB * kP; e += kNT) {
        const int pi = e / kP, x = e % kP;
        const int a = sm.ab[pi][0], b = sm.ab[pi][1];
        const double c = sm.cs[pi][0], s = sm.cs[pi][1];
        const double ga = sm.G[x][a], gb = sm.G[x][b];
        sm.G[x][a] = c * ga - s * gb;
        sm.G[x][b] = s * ga + c * gb;
        const double ja = sm.J[x][a], jb = sm.J[x][b];
        sm.J[x][a] = c * ja - s * jb;
        sm.J[x][b] = s * ja + c * jb;
      }
      __syncthreads();
    }
    if (tid == 0) sm.flag = 0;
    __syncthreads();
    if (off_exceeds(1e-15)) sm.flag = 1;
    __syncthreads();
    if (!sm.flag) break;
    __syncthreads();
  }

  // 3. X <- X J on the work matrix and on V
  apply_rotation(W, R, R, col, sm);
  apply_rotation(V, Cp, Cp, col, sm);
}

constexpr int kLdsDoubles = 19200;   // 150 KiB of LDS for the resident block pair
constexpr int kInnerLds = 1;         // sweeps over a block pair per visit

// rows a block pair of 2 KB columns can hold in LDS (with its 2KB x 2KB J)
constexpr int64_t lds_rows(int KB) { return (kLdsDoubles - 4 * KB * KB) / (2 * KB); }
// LDS column length for R rows: a multiple of the rows one pass of a column
// pair's threads covers (kNT / KB lanes, two rows each), zero past R
constexpr int64_t lds_padded_rows(int64_t R, int KB) {
  return (R + 2 * (kNT / KB) - 1) / (2 * (kNT / KB)) * (2 * (kNT / KB));
}

// x from another lane of the same 16-lane row (a DPP move; CTRL is the
// row-local lane pattern), both 32-bit halves
template <int CTRL>
__device__ __forceinline__ double dpp_move(double x) {
  const long long v = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)v, CTRL, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(v >> 32), CTRL, 0xf, 0xf, false);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned int)lo);
}

// sum over each 16-lane row, in every lane of the row: lane pairs (xor 1),
// quads (xor 2), mirrored half-rows, mirrored rows; each step adds the same
// two values in every lane it joins, so all lanes hold the same sum
__device__ __forceinline__ double row_sum(double x) {
  x += dpp_move<0xB1>(x);    // quad_perm [1, 0, 3, 2]
  x += dpp_move<0x4E>(x);    // quad_perm [2, 3, 0, 1]
  x += dpp_move<0x141>(x);   // row_half_mirror
  x += dpp_move<0x140>(x);   // row_mirror
  return x;
}

// Workgroup barrier for LDS data only: waits for this wave's LDS operations,
// not for its global loads in flight (a __syncthreads fence waits for both)
__device__ __forceinline__ void lds_barrier() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

template <int KB>
__global__ void __launch_bounds__(kNT) jacobi_lds_kernel(double* W, double* V, int64_t R, int64_t Cp, int nb,
                                                        int round, double tol, int* rotated, const int* perm) {
  constexpr int NC = 2 * KB;          // columns of the pair
  constexpr int TPP = kNT / KB;       // threads per column pair of a step (a power of two <= 256)
  __shared__ double lds[kLdsDoubles];
  __shared__ int any_rot;
  double* J = lds;                    // NC x NC, J[i * NC + j]
  double* X = lds + NC * NC;          // column c at X + c * Rp (16-byte aligned)
  const int Rp = (int)lds_padded_rows(R, KB);
  const int NI = Rp / (2 * TPP);      // two-row loads per lane over a column
  const int tid = threadIdx.x;
  // rows per thread per pass of the copies below: 32 loads in flight per
  // thread before their values are used (one load at a time waits out the
  // memory latency once per load)
  constexpr int U = NC >= 16 ? 1 : 16 / NC;
  int p, q;
  round_pair(nb, round, blockIdx.x, p, q);
  int64_t col[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) col[c] = perm[c < KB ? p * KB + c : q * KB + (c - KB)];
  // (loads past the last row read the last row again: no branch around them)
  for (int64_t r0 = 0; r0 < Rp; r0 += (int64_t)U * kNT) {
    double t[NC][U];
#pragma unroll
    for (int c = 0; c < NC; ++c)
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int64_t r = r0 + u * kNT + tid;
        t[c][u] = W[col[c] * R + (r < R ? r : R - 1)];
      }
#pragma unroll
    for (int c = 0; c < NC; ++c)
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int64_t r = r0 + u * kNT + tid;
        if (r < Rp) X[c * Rp + r] = r < R ? t[c][u] : 0.0;
      }
  }
  // the first U * kNT rows of the pair's V columns, loaded now: their latency
  // overlaps the rotations (the barriers below wait for LDS only)
  // (not for KB = 8, whose registers the rotations need)
  constexpr bool kPrefetch = NC <= 8;
  double vp[U][NC];
  if constexpr (kPrefetch) {
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        const int64_t r = u * kNT + tid;
        vp[u][c] = V[col[c] * Cp + (r < Cp ? r : Cp - 1)];
      }
  }
  for (int e = tid; e < NC * NC; e += kNT) J[e] = (e / NC) == (e % NC) ? 1.0 : 0.0;
  if (tid == 0) any_rot = 0;
  lds_barrier();

  const int pi = tid / TPP, lane = tid % TPP;   // column pair of the step, lane within it
  bool rotated_here = false;
  for (int sweep = 0; sweep < kInnerLds; ++sweep) {
    bool rot_sweep = false;
#pragma unroll 1
    for (int step = 0; step < NC - 1; ++step) {
      // the step's pairs: the circle method on NC columns (NC = 2: one pair)
      int a, b;
      if (NC == 2) {
        a = 0;
        b = 1;
      } else if (pi == 0) {
        a = NC - 1;
        b = step;
      } else {
        a = (step + pi) % (NC - 1);
        b = (step - pi + NC - 1) % (NC - 1);
      }
      if (a > b) {
        const int t = a;
        a = b;
        b = t;
      }
      const double2* xa = reinterpret_cast<const double2*>(X + a * Rp);
      const double2* xb = reinterpret_cast<const double2*>(X + b * Rp);
      double al = 0.0, be = 0.0, ga = 0.0;
#pragma unroll 4
      for (int i = 0; i < NI; ++i) {
        const double2 u = xa[i * TPP + lane], v = xb[i * TPP + lane];
        al += u.x * u.x + u.y * u.y;
        be += v.x * v.x + v.y * v.y;
        ga += u.x * v.x + u.y * v.y;
      }
      // sums over the pair's lanes: within each 16-lane row by DPP moves, then
      // across rows by lane exchanges (every lane ends with the same values)
      static_assert(TPP >= 32, "a column pair spans at least two rows of 16 lanes");
      al = row_sum(al);
      be = row_sum(be);
      ga = row_sum(ga);
#pragma unroll
      for (int o = 16; o < TPP && o < 64; o <<= 1) {
        al += __shfl_xor(al, o, 64);
        be += __shfl_xor(be, o, 64);
        ga += __shfl_xor(ga, o, 64);
      }
      if constexpr (TPP > 64) {
        // several wavefronts per pair: add the wavefront sums through LDS
        __shared__ double part[kNT / 64][3];
        const int wv = tid / 64;
        if ((tid & 63) == 0) {
          part[wv][0] = al;
          part[wv][1] = be;
          part[wv][2] = ga;
        }
        lds_barrier();
        const int w0 = (pi * TPP) / 64;
        al = be = ga = 0.0;
        for (int w = 0; w < TPP / 64; ++w) {
          al += part[w0 + w][0];
          be += part[w0 + w][1];
          ga += part[w0 + w][2];
        }
      }
      double c = 1.0, sn = 0.0;
      // |ga| > tol sqrt(al be), squared (ga^2 <= al be, so no new overflow)
      const bool rot = ga != 0.0 && ga * ga > (tol * tol) * (al * be);
      if (rot) {
        const double zeta = (be - al) / (2.0 * ga);
        const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
        c = rsqrt(1.0 + t * t);
        sn = t * c;
        rot_sweep = true;
        double2* wa = reinterpret_cast<double2*>(X + a * Rp);
        double2* wb = reinterpret_cast<double2*>(X + b * Rp);
#pragma unroll 4
        for (int i = 0; i < NI; ++i) {
          const double2 u = wa[i * TPP + lane], v = wb[i * TPP + lane];
          wa[i * TPP + lane] = make_double2(c * u.x - sn * v.x, c * u.y - sn * v.y);
          wb[i * TPP + lane] = make_double2(sn * u.x + c * v.x, sn * u.y + c * v.y);
        }
        for (int i = lane; i < NC; i += TPP) {
          const double u = J[i * NC + a], v = J[i * NC + b];
          J[i * NC + a] = c * u - sn * v;
          J[i * NC + b] = sn * u + c * v;
        }
      }
      lds_barrier();
    }
    if (rot_sweep) any_rot = 1;
    lds_barrier();
    const bool more = any_rot != 0;
    lds_barrier();
    if (tid == 0) any_rot = 0;
    if (!more) break;
    rotated_here = true;
    lds_barrier();
  }
  if (!rotated_here) {
    // already orthogonal: W and V unchanged (the V loads still in flight are
    // waited for before the wave ends)
    __builtin_amdgcn_s_waitcnt(0);
    return;
  }
  if (tid == 0) atomicAdd(rotated, 1);
  for (int c = 0; c < NC; ++c)
    for (int64_t r = tid; r < R; r += kNT) W[col[c] * R + r] = X[c * Rp + r];
  // V[:, cols] <- V[:, cols] J: U rows per thread at a time, each row's NC
  // values in registers, J read from LDS (every lane reads the same entry)
  for (int64_t r0 = 0; r0 < Cp; r0 += (int64_t)U * kNT) {
    // J stays in LDS for KB = 8 (its 256 entries would take 512 registers
    // if hoisted out of the loop)
    if constexpr (NC >= 16) asm volatile("" ::: "memory");
    double v[U][NC];
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        const int64_t r = r0 + u * kNT + tid;
        v[u][c] = kPrefetch && r0 == 0 ? vp[u][c] : V[col[c] * Cp + (r < Cp ? r : Cp - 1)];
      }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t r = r0 + u * kNT + tid;
      double o[NC];
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        double acc = 0.0;
#pragma unroll
        for (int i = 0; i < NC; ++i) acc += v[u][i] * J[i * NC + c];
        o[c] = acc;
      }
      if (r < Cp) {
#pragma unroll
        for (int c = 0; c < NC; ++c) V[col[c] * Cp + r] = o[c];
      }
    }
  }
}

__global__ void zero_int_kernel(int* p) { p[0] = 0; }

// X (C x Cp, column-major) = R^T for the upper triangle R of the factorised
// W (R x C, column-major): X[r, c] = R[c, r] for c <= r; zero above the
// diagonal of X and in the padding columns
__global__ void svd_x_from_r_kernel(const double* __restrict__ W, int64_t R, int64_t C, int64_t Cp, double* __restrict__ X) {
  const int64_t total = C * Cp;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = e % C, c = e / C;
    X[e] = (c < C && c <= r) ? W[r * R + c] : 0.0;
  }
}

// T (R x Cp, column-major) = [J diag(sigma); 0] with J the leading C x C
// block of the accumulated rotations V
__global__ void svd_precond_t_kernel(const double* __restrict__ V, const double* __restrict__ sigma, int64_t R,
                                     int64_t C, int64_t Cp, double* __restrict__ T) {
  const int64_t total = R * Cp;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = e % R, c = e / R;
    T[e] = (r < C && c < C) ? V[c * Cp + r] * sigma[c] : 0.0;
  }
}

// V (Cp x Cp) = the normalised columns of the converged X (zero for a zero
// column), the identity past C
__global__ void svd_precond_v_kernel(const double* __restrict__ X, const double* __restrict__ sigma, int64_t C,
                                     int64_t Cp, double* __restrict__ V) {
  const int64_t total = Cp * Cp;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = e % Cp, c = e / Cp;
    V[e] = c < C ? ((r < C && sigma[c] > 0.0) ? X[c * C + r] / sigma[c] : 0.0) : (r == c ? 1.0 : 0.0);
  }
}

__global__ void svd_copy_kernel(const double* __restrict__ src, double* __restrict__ dst, int64_t n) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
    dst[e] = src[e];
}

// sigma[c] = || W[:, c] ||_2, one 256-thread workgroup per column
__global__ void column_norm_kernel(const double* W, int64_t R, double* sigma) {
  __shared__ double part[kNT];
  const int64_t c = blockIdx.x;
  double s = 0.0;
  for (int64_t r = threadIdx.x; r < R; r += kNT) {
    const double x = W[c * R + r];
    s += x * x;
  }
  part[threadIdx.x] = s;
  __syncthreads();
  for (int w = kNT / 2; w >= 1; w >>= 1) {
    if ((int)threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) sigma[c] = sqrt(part[0]);
}

// order[t] = the column of the t-th largest singular value (ties: lower column first)
// one wavefront per column j: its lanes count the larger values (ties by
// index) over strided parts of sigma, then add their counts
__global__ void __launch_bounds__(256) rank_kernel(const double* sigma, int n, int* order) {
  const int lane = threadIdx.x & 63;
  const int nw = (int)((gridDim.x * blockDim.x) >> 6);
  for (int j = (int)((blockIdx.x * blockDim.x + threadIdx.x) >> 6); j < n; j += nw) {
    const double sj = sigma[j];
    int rank = 0;
    for (int i = lane; i < n; i += 64) {
      const double si = sigma[i];
      rank += (si > sj || (si == sj && i < j)) ? 1 : 0;
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) rank += __shfl_xor(rank, o, 64);
    if (lane == 0) order[rank] = j;
  }
}

// Truncation rule of Appendix A on the descending singular values s[0..kmax):
// k_count = min(kmax, max_sv) (max_sv <= 0: none), k_err = the smallest k with
// sum(s[k:]) <= max_err (max_err < 0: none), k = max(1, min(k_count, k_err)).
// The dropped sum is formed from the small end (smallest values first).
__global__ void truncate_kernel(const double* sigma, const int* order, int kmax, int max_sv, double max_err, int* k_out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  int k = kmax;
  if (max_sv > 0 && max_sv < k) k = max_sv;
  if (max_err >= 0.0) {
    double dropped = 0.0;   // sum of s[j..kmax)
    int kerr = kmax;
    for (int j = kmax - 1; j >= 0; --j) {
      dropped += sigma[order[j]];
      if (dropped <= max_err) kerr = j; else break;
    }
    if (kerr < k) k = kerr;
  }
  k_out[0] = k < 1 ? 1 : k;
}

// Output writer.  mode 0 (split_node): left = U sqrt(S), right = sqrt(S) V^T;
// mode 1 (full SVD): left = U, s = S, right = V^T.  U and V^T are read from
// the normalised columns of W (the longer side) and from V; which is which
// depends on `transposed`.  Every output is a strided view in the node's
// dtype with the new bond innermost in `left` and outermost in `right`.
struct OutView {
  void* p;
  int32_t dtype;
  int32_t n;                      // axes besides the new bond
  int64_t dim[TN_MAX_RANK], st[TN_MAX_RANK];
  int64_t kst;                    // stride of the new bond axis
};

__device__ inline void store_val(const OutView& o, int64_t off, double v) {
  if (o.dtype == TN_F64) static_cast<double*>(o.p)[off] = v;
  else static_cast<float*>(o.p)[off] = (float)v;
}

// U[i, t] or V[j, t] of A for sorted index t: from the column order[t] of W
// (normalised) or of the accumulated rotations
__device__ inline double long_side(const double* W, int64_t R, const double* sigma, int col, int64_t r) {
  const double s = sigma[col];
  return s > 0.0 ? W[(int64_t)col * R + r] / s : 0.0;
}

__global__ void write_factor_kernel(OutView o, int side, const double* W, const double* V, const double* sigma,
                                    const int* order, int64_t R, int64_t Cp, int transposed, int k, int mode) {
  // side 0: left factor [rows of A..., k]; side 1: right factor [k, cols of A...]
  int64_t m = 1;
  for (int a = 0; a < o.n; ++a) m *= o.dim[a];
  const int64_t total = m * k;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e / k;       // row of A (side 0) or column of A (side 1)
    const int t = (int)(e % k);
    const int col = order[t];
    const double s = sigma[col];
    // the singular vector of A's side `side`, entry i
    const bool from_w = (side == 0) != (transposed != 0);
    double x = from_w ? long_side(W, R, sigma, col, i) : V[(int64_t)col * Cp + i];
    if (mode == 0) x *= sqrt(s);
    int64_t off = t * o.kst;
    int64_t idx = i;
    for (int a = o.n - 1; a >= 0; --a) {
      const int64_t q = idx / o.dim[a];
      off += (idx - q * o.dim[a]) * o.st[a];
      idx = q;
    }
    store_val(o, off, x);
  }
}

// s (mode 1): rank 1 [k] or rank 2 [k, k] diagonal; trun_err[t] = s_sorted[k + t]
__global__ void write_values_kernel(OutView s_out, int s_rank, OutView tr_out, const double* sigma, const int* order,
                                    int k, int kmax) {
  const int64_t ns = s_out.p ? (s_rank == 2 ? (int64_t)k * k : k) : 0;
  const int64_t nt = tr_out.p ? (kmax - k) : 0;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < ns + nt; e += (int64_t)gridDim.x * blockDim.x) {
    if (e < ns) {
      if (s_rank == 2) {
        const int64_t i = e / k, j = e % k;
        store_val(s_out, i * s_out.st[0] + j * s_out.st[1], i == j ? sigma[order[i]] : 0.0);
      } else {
        store_val(s_out, e * s_out.st[0], sigma[order[e]]);
      }
    } else {
      const int64_t t = e - ns;
      store_val(tr_out, t * tr_out.st[0], sigma[order[k + t]]);
    }
  }
}

// ---------------------------------------------------------------------------
// host side

struct SvdGeom {
  int64_t ml, mr;        // rows (left legs) and columns (right legs) of A
  int64_t R, C, Cp;      // work matrix W: R x Cp, C = min(ml, mr) real columns
  int nb;                // column blocks (even)
  int kb;                // columns per block
  bool lds;              // block pairs resident in LDS (one-sided rotations)
  int transposed;        // W = A^T
  bool precond;          // Jacobi on R^T from a Householder QR of W (see the decompose call)
  size_t w_off, v_off, sigma_off, order_off, perm_off, ctl_off, x_off, t_off, tau_off, tf_off, total;
};

size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

int32_t svd_geometry(const tn_tensor* a, int32_t n_left, SvdGeom& g) {
  TN_TRY(check_tensor(a, "node", -1));
  if (a->rank < 2) return fail(TN_ERR_INVALID_ARGUMENT, "a node of rank %d cannot be split", a->rank);
  if (n_left < 1 || n_left >= a->rank)
    return fail(TN_ERR_INVALID_ARGUMENT, "n_left = %d: both effective legs need at least one axis", n_left);
  g.ml = g.mr = 1;
  for (int i = 0; i < n_left; ++i) g.ml *= a->shape[i];
  for (int i = n_left; i < a->rank; ++i) g.mr *= a->shape[i];
  g.transposed = g.ml < g.mr;
  g.R = std::max(g.ml, g.mr);
  g.C = std::min(g.ml, g.mr);
  if (g.C > 16384) return fail(TN_ERR_UNSUPPORTED, "the shorter effective leg (%lld) exceeds 16384", (long long)g.C);
  // Block width: a sweep is nb - 1 rounds (nb ~ C / KB), each one launch
  // whose pairs run side by side and whose work per pair grows like KB^2 R.
  // Modelled sweep time: rounds x (13 us + 0.72 us x KB^2 x R / 1000), plus
  // 3 us a round for KB = 1 (its pair spans four wavefronts), fitted to the
  // LDS kernel on gfx950 at R = 1000 (17, 16, 25 and 57 us a round for KB =
  // 1, 2, 4, 8); the cheapest width whose pair fits in LDS is taken.
  // QR preconditioning (see the decompose call) runs the sweeps on a C x C
  // matrix instead of the R x C one
  g.precond = householder_qr_fits(g.R) && g.C >= kPrecondMinCols;
  const int64_t jr = g.precond ? g.C : g.R;   // rows of the swept matrix
  g.kb = kB;   // Gram-matrix pair kernel
  double best = INFINITY;
  g.lds = false;
  for (int w : {8, 4, 2, 1}) {
    if (lds_padded_rows(jr, w) > lds_rows(w)) continue;
    // width 8's fifteen dependent steps a round cost more than the model
    // holds at a few hundred rows and up: width 4 measured faster at 512
    // rows (the chi = 256 DMRG split) and at 1000
    if (w == 8 && jr >= 384) continue;
    g.lds = true;
    int nbw = (int)((g.C + w - 1) / w);
    nbw = nbw < 2 ? 2 : nbw + (nbw % 2);
    const double t = (nbw - 1) * (13.0 + (w == 1 ? 3.0 : 0.0) + 0.72 * w * w * (double)jr / 1000.0);
    if (t < best) {
      best = t;
      g.kb = w;
    }
  }
  g.nb = (int)((g.C + g.kb - 1) / g.kb);
  if (g.nb < 2) g.nb = 2;
  if (g.nb % 2) g.nb += 1;
  g.Cp = (int64_t)g.nb * g.kb;
  size_t o = 0;
  g.w_off = o;
  o += al256((size_t)g.R * g.Cp * 8);
  g.v_off = o;
  o += al256((size_t)g.Cp * g.Cp * 8);
  g.sigma_off = o;
  o += al256((size_t)g.Cp * 8);
  g.order_off = o;
  o += al256((size_t)g.Cp * 4);
  g.perm_off = o;
  o += al256((size_t)g.Cp * 4);
  g.ctl_off = o;
  o += 256;
  // QR preconditioning: X = R^T (C x Cp), the Q product's target (R x Cp),
  // the reflectors' tau and triangular factors
  g.x_off = g.t_off = g.tau_off = g.tf_off = o;
  if (g.precond) {
    g.x_off = o;
    o += al256((size_t)g.C * g.Cp * 8);
    g.t_off = o;
    o += al256((size_t)g.R * g.Cp * 8);
    g.tau_off = o;
    o += al256((size_t)g.C * 8);
    g.tf_off = o;
    o += al256(householder_tf_doubles(g.C) * 8);
  }
  g.total = o;
  return TN_OK;
}

int32_t out_view(const tn_tensor* t, const char* name, int32_t dtype, OutView& o) {
  TN_TRY(check_tensor(t, name, dtype));
  std::memset(&o, 0, sizeof(o));
  o.p = t->data;
  o.dtype = t->dtype;
  return TN_OK;
}

// left [rows of A..., k] or right [k, cols of A...] against the node's legs
int32_t factor_view(const tn_tensor* t, const char* name, const tn_tensor* a, int32_t n_left, int side, int k,
                    OutView& o) {
  TN_TRY(out_view(t, name, a->dtype, o));
  const int nl = side == 0 ? n_left : a->rank - n_left;
  const int first = side == 0 ? 0 : n_left;
  if (t->rank != nl + 1) return fail(TN_ERR_SHAPE_MISMATCH, "%s must have rank %d", name, nl + 1);
  const int kax = side == 0 ? nl : 0;
  if (t->shape[kax] != k) return fail(TN_ERR_SHAPE_MISMATCH, "%s: the new bond must have extent %d", name, k);
  o.kst = t->stride[kax];
  o.n = nl;
  for (int q = 0; q < nl; ++q) {
    const int ax = side == 0 ? q : q + 1;
    if (t->shape[ax] != a->shape[first + q]) return fail(TN_ERR_SHAPE_MISMATCH, "%s: axis %d extent differs from the node", name, ax);
    o.dim[q] = t->shape[ax];
    o.st[q] = t->stride[ax];
  }
  if (has_internal_overlap(*t)) return fail(TN_ERR_INVALID_ARGUMENT, "%s maps two indices to one address", name);
  return TN_OK;
}

int32_t write_outputs(const tn_tensor* a, int32_t n_left, int32_t k, const tn_tensor* left, const tn_tensor* s,
                      const tn_tensor* right, const tn_tensor* trun_err, int mode, void* workspace, size_t ws_bytes,
                      void* stream) {
  SvdGeom g;
  TN_TRY(svd_geometry(a, n_left, g));
  if (!workspace || ws_bytes < g.total) return fail(TN_ERR_WORKSPACE_TOO_SMALL, "workspace needs %zu bytes", g.total);
  if (k < 1 || k > g.C) return fail(TN_ERR_INVALID_ARGUMENT, "k = %d outside 1..%lld", k, (long long)g.C);
  OutView lo, ro, so, to;
  TN_TRY(factor_view(left, "left", a, n_left, 0, k, lo));
  TN_TRY(factor_view(right, "right", a, n_left, 1, k, ro));
  std::memset(&so, 0, sizeof(so));
  std::memset(&to, 0, sizeof(to));
  int s_rank = 0;
  if (mode == 1) {
    TN_TRY(out_view(s, "s", a->dtype, so));
    s_rank = s->rank;
    if (!((s->rank == 1 && s->shape[0] == k) || (s->rank == 2 && s->shape[0] == k && s->shape[1] == k)))
      return fail(TN_ERR_SHAPE_MISMATCH, "s must be [k] or [k, k] with k = %d", k);
    so.st[0] = s->stride[0];
    so.st[1] = s->rank == 2 ? s->stride[1] : 0;
  }
  if (trun_err) {
    TN_TRY(out_view(trun_err, "trun_err", a->dtype, to));
    if (trun_err->rank != 1 || trun_err->shape[0] != g.C - k)
      return fail(TN_ERR_SHAPE_MISMATCH, "trun_err must be [%lld] (the dropped values)", (long long)(g.C - k));
    to.st[0] = trun_err->stride[0];
  }
  const tn_tensor* outs[4] = {left, right, mode == 1 ? s : nullptr, trun_err};
  for (int i = 0; i < 4; ++i) {
    if (!outs[i]) continue;
    if (overlaps(*outs[i], *a)) return fail(TN_ERR_ALIASING, "an output overlaps the node");
    for (int j = i + 1; j < 4; ++j)
      if (outs[j] && overlaps(*outs[i], *outs[j])) return fail(TN_ERR_ALIASING, "two outputs overlap");
  }
  char* ws = static_cast<char*>(workspace);
  const double* W = reinterpret_cast<const double*>(ws + g.w_off);
  const double* V = reinterpret_cast<const double*>(ws + g.v_off);
  const double* sigma = reinterpret_cast<const double*>(ws + g.sigma_off);
  const int* order = reinterpret_cast<const int*>(ws + g.order_off);
  hipStream_t st = static_cast<hipStream_t>(stream);
  auto blocks = [](int64_t n) { return (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 8192)); };
  hipLaunchKernelGGL(write_factor_kernel, dim3(blocks(g.ml * k)), dim3(256), 0, st, lo, 0, W, V, sigma, order, g.R,
                     g.Cp, g.transposed, k, mode);
  hipLaunchKernelGGL(write_factor_kernel, dim3(blocks(g.mr * k)), dim3(256), 0, st, ro, 1, W, V, sigma, order, g.R,
                     g.Cp, g.transposed, k, mode);
  const int64_t nv = (mode == 1 ? (s_rank == 2 ? (int64_t)k * k : k) : 0) + (trun_err ? g.C - k : 0);
  if (nv > 0)
    hipLaunchKernelGGL(write_values_kernel, dim3(blocks(nv)), dim3(256), 0, st, so, s_rank, to, sigma, order, k,
                       (int)g.C);
  return hip_check(hipGetLastError(), "split node outputs");
}

}  // namespace

}  // namespace tn

using namespace tn;

extern "C" {

int32_t tn_split_node_workspace(const tn_tensor* a, int32_t n_left, size_t* bytes) {
  if (!bytes) return fail(TN_ERR_INVALID_ARGUMENT, "bytes is NULL");
  SvdGeom g;
  TN_TRY(svd_geometry(a, n_left, g));
  *bytes = g.total;
  return TN_OK;
}

int32_t tn_split_node_decompose(const tn_tensor* a, int32_t n_left, int32_t max_singular_values,
                                double max_truncation_err, int32_t* k, int32_t* sweeps, void* workspace,
                                size_t ws_bytes, void* stream) {
  SvdGeom g;
  TN_TRY(svd_geometry(a, n_left, g));
  if (!k) return fail(TN_ERR_INVALID_ARGUMENT, "k is NULL");
  if (!workspace || ws_bytes < g.total) return fail(TN_ERR_WORKSPACE_TOO_SMALL, "workspace needs %zu bytes", g.total);
  if (std::isnan(max_truncation_err)) return fail(TN_ERR_INVALID_ARGUMENT, "max_truncation_err is NaN");
  {
    tn_tensor wsv = make_view(workspace, TN_F64, {(int64_t)(g.total / 8)});
    if (overlaps(*a, wsv)) return fail(TN_ERR_ALIASING, "the workspace overlaps the node");
  }
  MatView mv;
  std::memset(&mv, 0, sizeof(mv));
  mv.p = a->data;
  mv.dtype = a->dtype;
  mv.nr = n_left;
  mv.nc = a->rank - n_left;
  for (int i = 0; i < n_left; ++i) {
    mv.rdim[i] = a->shape[i];
    mv.rst[i] = a->stride[i];
  }
  for (int i = n_left; i < a->rank; ++i) {
    mv.cdim[i - n_left] = a->shape[i];
    mv.cst[i - n_left] = a->stride[i];
  }
  char* ws = static_cast<char*>(workspace);
  double* W = reinterpret_cast<double*>(ws + g.w_off);
  double* V = reinterpret_cast<double*>(ws + g.v_off);
  double* sigma = reinterpret_cast<double*>(ws + g.sigma_off);
  int* order = reinterpret_cast<int*>(ws + g.order_off);
  int* ctl = reinterpret_cast<int*>(ws + g.ctl_off);   // [0]: pairs rotated in the sweep, [1]: k
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int64_t ng = g.R * g.Cp + g.Cp * g.Cp;
  hipLaunchKernelGGL(svd_gather_kernel, dim3((unsigned)std::min<int64_t>((ng + 255) / 256, 16384)), dim3(256), 0, st,
                     mv, g.transposed, g.R, g.C, g.Cp, W, V);
  TN_TRY(hip_check(hipGetLastError(), "svd gather"));
  int done_sweeps = 0;
  int* perm = reinterpret_cast<int*>(ws + g.perm_off);
  // one-sided Jacobi sweeps on the columns of M (rows x Cp), rotations
  // accumulated in V, until a sweep rotates no pair
  auto sweep_until_done = [&](double* M, int64_t rows) -> int32_t {
    // pairs count as orthogonal when |g_ij| <= tol sqrt(g_ii g_jj): a few
    // roundings of a dot product of length `rows`
    const double tol = 8.0 * std::sqrt((double)rows) * 2.220446049250313e-16;
    for (int sw = 0; sw < kMaxSweeps; ++sw) {
      // columns in descending order of their norms: the blocks of a sweep then
      // pair columns of similar size first (fewer sweeps on graded spectra)
      hipLaunchKernelGGL(column_norm_kernel, dim3((unsigned)g.Cp), dim3(kNT), 0, st, M, rows, sigma);
      hipLaunchKernelGGL(rank_kernel, dim3((unsigned)((g.Cp + 3) / 4)), dim3(256), 0, st, sigma, (int)g.Cp, perm);
      hipLaunchKernelGGL(zero_int_kernel, dim3(1), dim3(1), 0, st, ctl);
      for (int r = 0; r < g.nb - 1; ++r) {
        const dim3 grid(g.nb / 2), blk(kNT);
        if (!g.lds)
          hipLaunchKernelGGL(jacobi_pair_kernel, grid, blk, 0, st, M, V, rows, g.Cp, g.nb, r, tol, ctl, perm);
        else if (g.kb == 8)
          hipLaunchKernelGGL(jacobi_lds_kernel<8>, grid, blk, 0, st, M, V, rows, g.Cp, g.nb, r, tol, ctl, perm);
        else if (g.kb == 4)
          hipLaunchKernelGGL(jacobi_lds_kernel<4>, grid, blk, 0, st, M, V, rows, g.Cp, g.nb, r, tol, ctl, perm);
        else if (g.kb == 2)
          hipLaunchKernelGGL(jacobi_lds_kernel<2>, grid, blk, 0, st, M, V, rows, g.Cp, g.nb, r, tol, ctl, perm);
        else
          hipLaunchKernelGGL(jacobi_lds_kernel<1>, grid, blk, 0, st, M, V, rows, g.Cp, g.nb, r, tol, ctl, perm);
      }
      TN_TRY(hip_check(hipGetLastError(), "jacobi sweep"));
      int rotated = 0;
      TN_TRY(hip_check(hipMemcpyAsync(&rotated, ctl, sizeof(int), hipMemcpyDeviceToHost, st), "read sweep counter"));
      TN_TRY(hip_check(hipStreamSynchronize(st), "sweep sync"));
      done_sweeps = sw + 1;
      if (rotated == 0) break;
    }
    return TN_OK;
  };
  if (!g.precond) {
    TN_TRY(sweep_until_done(W, g.R));
  } else {
    // Preconditioning (Drmac and Veselic): W = Q R by Householder QR, then
    // one-sided Jacobi on X = R^T, whose columns are far closer to
    // orthogonal on graded spectra (measured on 1000 x 1000, e^(-i/40): 41
    // sweeps on W, a few on X).  X J = V_W S and J = Q^T U_W for W = U_W S
    // V_W^T, so U_W S = Q [J S; 0] and V_W = X J S^-1: the same W (columns
    // U S) and V as the sweeps on W leave.
    double* X = reinterpret_cast<double*>(ws + g.x_off);
    double* T = reinterpret_cast<double*>(ws + g.t_off);
    double* tau = reinterpret_cast<double*>(ws + g.tau_off);
    double* tf = reinterpret_cast<double*>(ws + g.tf_off);
    const unsigned gx = (unsigned)std::min<int64_t>((g.R * g.Cp + 255) / 256, 16384);
    TN_TRY(householder_qr(W, (int)g.R, (int)g.C, tau, tf, st));
    hipLaunchKernelGGL(svd_x_from_r_kernel, dim3(gx), dim3(256), 0, st, W, g.R, g.C, g.Cp, X);
    TN_TRY(hip_check(hipGetLastError(), "svd precondition"));
    TN_TRY(sweep_until_done(X, g.C));
    hipLaunchKernelGGL(column_norm_kernel, dim3((unsigned)g.Cp), dim3(kNT), 0, st, X, g.C, sigma);
    hipLaunchKernelGGL(svd_precond_t_kernel, dim3(gx), dim3(256), 0, st, V, sigma, g.R, g.C, g.Cp, T);
    hipLaunchKernelGGL(svd_precond_v_kernel, dim3(gx), dim3(256), 0, st, X, sigma, g.C, g.Cp, V);
    TN_TRY(hip_check(hipGetLastError(), "svd precondition"));
    TN_TRY(householder_apply_q(W, (int)g.R, (int)g.C, tf, T, (int)g.C, st));
    hipLaunchKernelGGL(svd_copy_kernel, dim3(gx), dim3(256), 0, st, T, W, g.R * g.Cp);
    TN_TRY(hip_check(hipGetLastError(), "svd precondition"));
  }
  hipLaunchKernelGGL(column_norm_kernel, dim3((unsigned)g.Cp), dim3(kNT), 0, st, W, g.R, sigma);
  hipLaunchKernelGGL(rank_kernel, dim3((unsigned)((g.Cp + 3) / 4)), dim3(256), 0, st, sigma, (int)g.Cp, order);
  hipLaunchKernelGGL(truncate_kernel, dim3(1), dim3(64), 0, st, sigma, order, (int)g.C, max_singular_values,
                     max_truncation_err, ctl + 1);
  TN_TRY(hip_check(hipGetLastError(), "singular values"));
  int kk = 0;
  TN_TRY(hip_check(hipMemcpyAsync(&kk, ctl + 1, sizeof(int), hipMemcpyDeviceToHost, st), "read k"));
  TN_TRY(hip_check(hipStreamSynchronize(st), "svd sync"));
  *k = kk;
  if (sweeps) *sweeps = done_sweeps;
  return TN_OK;
}

int32_t tn_split_node(const tn_tensor* a, int32_t n_left, int32_t k, tn_tensor* left, tn_tensor* right,
                      tn_tensor* trun_err, void* workspace, size_t ws_bytes, void* stream) {
  return write_outputs(a, n_left, k, left, nullptr, right, trun_err, 0, workspace, ws_bytes, stream);
}

int32_t tn_split_node_full_svd(const tn_tensor* a, int32_t n_left, int32_t k, tn_tensor* u, tn_tensor* s,
                               tn_tensor* vh, tn_tensor* trun_err, void* workspace, size_t ws_bytes, void* stream) {
  if (!s) return fail(TN_ERR_INVALID_ARGUMENT, "s is NULL");
  return write_outputs(a, n_left, k, u, s, vh, trun_err, 1, workspace, ws_bytes, stream);
}

}  // extern "C"
