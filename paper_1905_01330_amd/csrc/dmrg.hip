// Two-site DMRG update on the GPU: the effective Hamiltonian of two
// neighbouring sites (section III.B names DMRG as the algorithm that splits
// nodes) and its lowest eigenpair by Lanczos.  The split of the eigenvector
// back into two sites is tn_split_node.
//
// (H_eff theta)[a', t1, t2, b'] =
//     sum L[a', u, a] W1[u, v, t1, s1] W2[v, x, t2, s2] R[b', x, b] theta[a, s1, s2, b]
// is one five-node network contracted by the ncon driver in the order
// L-theta, W1, W2, R (every step a tiled contraction on the matrix cores).
//
// Lanczos with full reorthogonalisation: the Krylov vectors are FP32, every
// dot product is accumulated in FP64 over a fixed tree (deterministic), and
// every scalar (the tridiagonal T, the Gram-Schmidt coefficients) stays in
// device memory, so a restart is a sequence of launches with no host
// synchronisation.  Each new vector is made orthogonal to all previous ones
// by classical Gram-Schmidt applied twice.  When the new residual is below
// kBreakdown of |H v_j| the Krylov space is exhausted: later vectors are
// zero and T is cut there.  T's lowest eigenpair comes from cyclic Jacobi in
// one workgroup; the Ritz vector starts the next restart.
#include <cmath>
#include <cstring>
#include <vector>

#include "internal.h"

namespace tn {

namespace {

constexpr int kMaxKry = 32;       // Krylov vectors per restart
constexpr int kDotBlocks = 256;   // partial sums per dot product
constexpr int kDotThreads = 256;
constexpr double kBreakdown = 1e-5;

// device scalars (doubles)
struct Scal {
  double alpha[kMaxKry], beta[kMaxKry], nraw[kMaxKry], coef[kMaxKry + 1], y[kMaxKry], tmp[4], eval, resid;
};

// part[i * G + g] = partial sum of V_i . w over the grid-stride slice of block g
__global__ void __launch_bounds__(kDotThreads) mdot_partial_kernel(const float* V, int64_t ld, const float* w,
                                                                   int64_t n, double* part) {
  __shared__ double red[kDotThreads];
  const int i = blockIdx.y, G = gridDim.x;
  const float* v = V + (int64_t)i * ld;
  double s = 0.0;
  for (int64_t e = (int64_t)blockIdx.x * kDotThreads + threadIdx.x; e < n; e += (int64_t)G * kDotThreads)
    s += (double)v[e] * (double)w[e];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = kDotThreads / 2; o >= 1; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[(int64_t)i * G + blockIdx.x] = red[0];
}

// out[i] = sum_g part[i * G + g] (fixed order); mode 1 also sets alpha[j] = out[j],
// mode 2 adds it
__global__ void mdot_finish_kernel(const double* part, int G, int count, double* out, double* alpha, int j, int mode) {
  const int i = threadIdx.x;
  if (i >= count) return;
  double s = 0.0;
  for (int g = 0; g < G; ++g) s += part[(int64_t)i * G + g];
  out[i] = s;
  if (i == j && mode == 1) alpha[j] = s;
  if (i == j && mode == 2) alpha[j] += s;
}

// w <- w - sum_{i < count} coef[i] V_i
__global__ void sub_combo_kernel(float* w, const float* V, int64_t ld, int count, const double* coef, int64_t n) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    double acc = (double)w[e];
    for (int i = 0; i < count; ++i) acc -= coef[i] * (double)V[(int64_t)i * ld + e];
    w[e] = (float)acc;
  }
}

// vout = w / sqrt(nrm2) unless sqrt(nrm2) <= rel * sqrt(ref) (then zero);
// beta_out (nullable) receives the norm or 0
__global__ void normalize_kernel(float* vout, const float* w, int64_t n, const double* nrm2, const double* ref,
                                 double rel, double* beta_out) {
  const double b = sqrt(nrm2[0]);
  const bool dead = !(b > rel * (ref ? sqrt(ref[0]) : 0.0)) || !(b > 0.0);
  const double inv = dead ? 0.0 : 1.0 / b;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
    vout[e] = (float)((double)w[e] * inv);
  if (beta_out && blockIdx.x == 0 && threadIdx.x == 0) beta_out[0] = dead ? 0.0 : b;
}

// out = sum_{j < m} y[j] V_j
__global__ void ritz_kernel(float* out, const float* V, int64_t ld, int m, const double* y, int64_t n) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    double acc = 0.0;
    for (int j = 0; j < m; ++j) acc += y[j] * (double)V[(int64_t)j * ld + e];
    out[e] = (float)acc;
  }
}

// r = w - eval * theta, written into w
__global__ void residual_kernel(float* w, const float* theta, const double* eval, int64_t n) {
  const double ev = eval[0];
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
    w[e] = (float)((double)w[e] - ev * (double)theta[e]);
}

__global__ void sqrt_to_kernel(const double* x, double* out) { out[0] = sqrt(x[0]); }

__global__ void energy_out_kernel(const Scal* sc, double* out2) {
  out2[0] = sc->eval;
  out2[1] = sc->resid;
}

// Lowest eigenpair of the symmetric tridiagonal T (alpha on the diagonal,
// beta beside it) of order m, cut after the first zero beta.  Cyclic Jacobi
// (Golub and Van Loan 8.5) on the dense matrix, padded to kMaxKry with a
// diagonal that is never the lowest.  One workgroup of 256 threads.
__global__ void __launch_bounds__(256) tridiag_min_kernel(const double* alpha, const double* beta, int m, double* y,
                                                         double* eval) {
  constexpr int P = kMaxKry;
  __shared__ double T[P][P + 1];
  __shared__ double Z[P][P + 1];
  __shared__ double cs[P / 2][2];
  __shared__ int ab[P / 2][2];
  __shared__ int m_eff;
  __shared__ double big;
  __shared__ int rotated;
  __shared__ double nrm;
  const int tid = threadIdx.x;
  if (tid == 0) {
    int me = m;
    for (int j = 0; j < m - 1; ++j)
      if (beta[j] == 0.0) {
        me = j + 1;
        break;
      }
    m_eff = me;
    double s = 0.0;
    for (int j = 0; j < me; ++j) s += fabs(alpha[j]) + (j + 1 < me ? 2.0 * fabs(beta[j]) : 0.0);
    nrm = s;                 // bounds |T| of the kept block from above
    big = 4.0 * (s + 1.0);   // above every eigenvalue of the kept block (Gershgorin)
  }
  __syncthreads();
  for (int e = tid; e < P * P; e += 256) {
    const int i = e / P, j = e % P;
    double v = 0.0;
    if (i < m_eff && j < m_eff) {
      if (i == j) v = alpha[i];
      else if (j == i + 1) v = beta[i];
      else if (i == j + 1) v = beta[j];
    } else if (i == j) {
      v = big + i;
    }
    T[i][j] = v;
    Z[i][j] = i == j ? 1.0 : 0.0;
  }
  __syncthreads();
  // sweeps until one rotates no pair (at most 20): a pair counts as
  // diagonal once |T_ab| <= 2^-60 |T|, which moves no eigenvalue by more
  // than that
  const double thr = 0x1p-60 * nrm;
  for (int sweep = 0; sweep < 20; ++sweep) {
    if (tid == 0) rotated = 0;
    __syncthreads();
    for (int step = 0; step < P - 1; ++step) {
      if (tid < P / 2) {
        int a, b;
        if (tid == 0) {
          a = P - 1;
          b = step;
        } else {
          a = (step + tid) % (P - 1);
          b = (step - tid + P - 1) % (P - 1);
        }
        if (a > b) {
          const int t = a;
          a = b;
          b = t;
        }
        const double app = T[a][a], aqq = T[b][b], apq = T[a][b];
        double c = 1.0, s = 0.0;
        if (fabs(apq) > thr) {
          rotated = 1;
          const double tau = (aqq - app) / (2.0 * apq);
          const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
          c = 1.0 / sqrt(1.0 + t * t);
          s = t * c;
        }
        cs[tid][0] = c;
        cs[tid][1] = s;
        ab[tid][0] = a;
        ab[tid][1] = b;
      }
      __syncthreads();
      for (int e = tid; e < (P / 2) * P; e += 256) {
        const int pi = e / P, x = e % P;
        const int a = ab[pi][0], b = ab[pi][1];
        const double c = cs[pi][0], s = cs[pi][1];
        const double ga = T[a][x], gb = T[b][x];
        T[a][x] = c * ga - s * gb;
        T[b][x] = s * ga + c * gb;
      }
      __syncthreads();
      for (int e = tid; e < (P / 2) * P; e += 256) {
        const int pi = e / P, x = e % P;
        const int a = ab[pi][0], b = ab[pi][1];
        const double c = cs[pi][0], s = cs[pi][1];
        const double ga = T[x][a], gb = T[x][b];
        T[x][a] = c * ga - s * gb;
        T[x][b] = s * ga + c * gb;
        const double za = Z[x][a], zb = Z[x][b];
        Z[x][a] = c * za - s * zb;
        Z[x][b] = s * za + c * zb;
      }
      __syncthreads();
    }
    if (rotated == 0) break;   // read by every thread after the last barrier
    __syncthreads();           // before thread 0 clears it for the next sweep
  }
  if (tid == 0) {
    int best = 0;
    for (int i = 1; i < P; ++i)
      if (T[i][i] < T[best][best]) best = i;
    eval[0] = T[best][best];
    // sign: largest component positive (any sign is an eigenvector)
    int im = 0;
    for (int i = 1; i < m; ++i)
      if (fabs(Z[i][best]) > fabs(Z[im][best])) im = i;
    const double sg = Z[im][best] < 0.0 ? -1.0 : 1.0;
    for (int i = 0; i < m; ++i) y[i] = i < m_eff ? sg * Z[i][best] : 0.0;
  }
}

// ---------------------------------------------------------------------------
// host side

struct Heff {
  tn_tensor nodes[5];
  int32_t labels[18];
  int32_t offsets[6];
  int32_t order[7];
  int64_t n;            // elements of theta
  int64_t shape[4];     // theta [Dl, d1, d2, Dr]
};

// L: a'=-1 u=1 a=2 | theta: a=2 s1=3 s2=4 b=5 | W1: u=1 v=6 t1=-2 s1=3 |
// W2: v=6 x=7 t2=-3 s2=4 | R: b'=-4 x=7 b=5; contraction order 2, 1, 6, 7
int32_t heff_setup(const tn_tensor* L, const tn_tensor* R, const tn_tensor* w1, const tn_tensor* w2,
                   const tn_tensor* theta_shape_src, Heff& h) {
  TN_TRY(check_tensor(L, "L", TN_F32));
  TN_TRY(check_tensor(R, "R", TN_F32));
  TN_TRY(check_tensor(w1, "w1", TN_F32));
  TN_TRY(check_tensor(w2, "w2", TN_F32));
  TN_TRY(check_tensor(theta_shape_src, "theta", TN_F32));
  if (L->rank != 3 || R->rank != 3 || w1->rank != 4 || w2->rank != 4 || theta_shape_src->rank != 4)
    return fail(TN_ERR_SHAPE_MISMATCH, "need L, R of rank 3, w1, w2 and theta of rank 4");
  const tn_tensor& t = *theta_shape_src;
  if (L->shape[0] != t.shape[0] || L->shape[2] != t.shape[0] || R->shape[0] != t.shape[3] || R->shape[2] != t.shape[3])
    return fail(TN_ERR_SHAPE_MISMATCH, "L must be [Dl, wl, Dl] and R [Dr, wr, Dr] for theta [Dl, d1, d2, Dr]");
  if (w1->shape[0] != L->shape[1] || w1->shape[1] != w2->shape[0] || w2->shape[1] != R->shape[1])
    return fail(TN_ERR_SHAPE_MISMATCH, "operator bonds differ (L, w1, w2, R)");
  if (w1->shape[2] != t.shape[1] || w1->shape[3] != t.shape[1] || w2->shape[2] != t.shape[2] || w2->shape[3] != t.shape[2])
    return fail(TN_ERR_SHAPE_MISMATCH, "physical dimensions of w1, w2 and theta differ");
  h.nodes[0] = *L;
  h.nodes[1] = t;
  h.nodes[2] = *w1;
  h.nodes[3] = *w2;
  h.nodes[4] = *R;
  const int32_t lab[18] = {-1, 1, 2, 2, 3, 4, 5, 1, 6, -2, 3, 6, 7, -3, 4, -4, 7, 5};
  std::memcpy(h.labels, lab, sizeof(lab));
  const int32_t off[6] = {0, 3, 7, 11, 15, 18};
  std::memcpy(h.offsets, off, sizeof(off));
  // every connected label once: contracting 1 also contracts 3, 6 also 4, 7 also 5
  const int32_t ord[7] = {2, 1, 3, 6, 4, 7, 5};
  std::memcpy(h.order, ord, sizeof(ord));
  h.n = 1;
  for (int i = 0; i < 4; ++i) {
    h.shape[i] = t.shape[i];
    h.n *= t.shape[i];
  }
  return TN_OK;
}

}  // namespace

}  // namespace tn

using namespace tn;

namespace tn {
namespace {

struct DmrgLayout {
  size_t net, v, w, part, sc, total;
  size_t net_bytes;
  int64_t ld;   // floats between Krylov vectors
};

int32_t dmrg_layout(Heff& h, int32_t krylov, DmrgLayout& d) {
  if (krylov < 2 || krylov > kMaxKry) return fail(TN_ERR_INVALID_ARGUMENT, "krylov must be in 2..%d", kMaxKry);
  size_t nb = 0;
  TN_TRY(tn_contract_network_workspace(5, h.nodes, h.labels, h.offsets, 7, h.order, &nb));
  auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
  d.ld = (h.n + 63) & ~(int64_t)63;
  d.net_bytes = nb;
  size_t o = 0;
  d.net = o;
  o += al(nb);
  d.v = o;
  o += al((size_t)(kMaxKry + 1) * d.ld * 4);
  d.w = o;
  o += al((size_t)d.ld * 4);
  d.part = o;
  o += al((size_t)(kMaxKry + 1) * kDotBlocks * 8);
  d.sc = o;
  o += al(sizeof(Scal));
  d.total = o;
  return TN_OK;
}

tn_tensor vec_view(float* p, const Heff& h) {
  return contiguous_view(p, TN_F32, 4, h.shape);
}

}  // namespace
}  // namespace tn

extern "C" {

int32_t tn_dmrg_workspace(const tn_tensor* L, const tn_tensor* R, const tn_tensor* w1, const tn_tensor* w2,
                          const tn_tensor* theta, int32_t krylov, size_t* bytes) {
  if (!bytes) return fail(TN_ERR_INVALID_ARGUMENT, "bytes is NULL");
  Heff h;
  TN_TRY(heff_setup(L, R, w1, w2, theta, h));
  DmrgLayout d;
  TN_TRY(dmrg_layout(h, krylov, d));
  *bytes = d.total;
  return TN_OK;
}

int32_t tn_dmrg_apply_heff(const tn_tensor* L, const tn_tensor* R, const tn_tensor* w1, const tn_tensor* w2,
                           const tn_tensor* theta, tn_tensor* out, void* workspace, size_t ws_bytes, int32_t prec,
                           void* stream) {
  Heff h;
  TN_TRY(heff_setup(L, R, w1, w2, theta, h));
  TN_TRY(check_tensor(out, "out", TN_F32));
  for (int i = 0; i < 4; ++i)
    if (out->rank != 4 || out->shape[i] != h.shape[i]) return fail(TN_ERR_SHAPE_MISMATCH, "out must have theta's shape");
  size_t nb = 0;
  TN_TRY(tn_contract_network_workspace(5, h.nodes, h.labels, h.offsets, 7, h.order, &nb));
  return tn_contract_network(5, h.nodes, h.labels, h.offsets, 7, h.order, out, workspace, ws_bytes, prec, stream);
}

int32_t tn_dmrg_eigensolve(const tn_tensor* L, const tn_tensor* R, const tn_tensor* w1, const tn_tensor* w2,
                           tn_tensor* theta, int32_t krylov, int32_t restarts, double* out2, void* workspace,
                           size_t ws_bytes, int32_t prec, void* stream) {
  Heff h;
  TN_TRY(heff_setup(L, R, w1, w2, theta, h));
  if (!out2) return fail(TN_ERR_INVALID_ARGUMENT, "out2 is NULL");
  if (restarts < 1) return fail(TN_ERR_INVALID_ARGUMENT, "restarts must be >= 1");
  if (prec < 0 || prec > 3) return fail(TN_ERR_UNSUPPORTED, "unknown precision %d", prec);
  {
    int64_t st = 1;
    for (int q = 3; q >= 0; --q) {
      if (theta->stride[q] != st) return fail(TN_ERR_UNSUPPORTED, "theta must be contiguous");
      st *= theta->shape[q];
    }
  }
  DmrgLayout d;
  TN_TRY(dmrg_layout(h, krylov, d));
  if (!workspace || ws_bytes < d.total) return fail(TN_ERR_WORKSPACE_TOO_SMALL, "workspace needs %zu bytes", d.total);
  for (int i = 0; i < 5; ++i)
    if (i != 1 && overlaps(*theta, h.nodes[i])) return fail(TN_ERR_ALIASING, "theta overlaps an operand");
  const int m = (int)std::min<int64_t>(krylov, h.n);
  hipStream_t st = static_cast<hipStream_t>(stream);
  char* ws = static_cast<char*>(workspace);
  void* net = ws + d.net;
  float* V = reinterpret_cast<float*>(ws + d.v);
  float* w = reinterpret_cast<float*>(ws + d.w);
  double* part = reinterpret_cast<double*>(ws + d.part);
  Scal* sc = reinterpret_cast<Scal*>(ws + d.sc);
  float* th = static_cast<float*>(theta->data);
  const int64_t n = h.n;
  const unsigned eb = (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 4096));
  const int G = (int)std::max<int64_t>(1, std::min<int64_t>(kDotBlocks, (n + 4095) / 4096));
  auto mdot = [&](const float* Vb, int count, const float* x, double* out, double* alpha, int j, int mode) {
    hipLaunchKernelGGL(mdot_partial_kernel, dim3(G, count), dim3(kDotThreads), 0, st, Vb, d.ld, x, n, part);
    hipLaunchKernelGGL(mdot_finish_kernel, dim3(1), dim3(64), 0, st, part, G, count, out, alpha, j, mode);
  };
  auto apply_h = [&](float* x, float* y) -> int32_t {
    h.nodes[1] = vec_view(x, h);
    tn_tensor o = vec_view(y, h);
    return tn_contract_network(5, h.nodes, h.labels, h.offsets, 7, h.order, &o, net, d.net_bytes, prec, stream);
  };
  // v_0 = theta / |theta|
  mdot(th, 1, th, sc->tmp, nullptr, 0, 0);
  hipLaunchKernelGGL(normalize_kernel, dim3(eb), dim3(256), 0, st, V, th, n, sc->tmp, nullptr, 0.0, nullptr);
  for (int rs = 0; rs < restarts; ++rs) {
    for (int j = 0; j < m; ++j) {
      float* vj = V + (int64_t)j * d.ld;
      TN_TRY(apply_h(vj, w));
      mdot(w, 1, w, sc->nraw + j, nullptr, 0, 0);
      // classical Gram-Schmidt against v_0 .. v_j, twice; alpha_j = the v_j coefficients
      for (int pass = 0; pass < 2; ++pass) {
        mdot(V, j + 1, w, sc->coef, sc->alpha, j, pass == 0 ? 1 : 2);
        hipLaunchKernelGGL(sub_combo_kernel, dim3(eb), dim3(256), 0, st, w, V, d.ld, j + 1, sc->coef, n);
      }
      mdot(w, 1, w, sc->tmp, nullptr, 0, 0);
      hipLaunchKernelGGL(normalize_kernel, dim3(eb), dim3(256), 0, st, V + (int64_t)(j + 1) * d.ld, w, n, sc->tmp,
                         sc->nraw + j, kBreakdown, sc->beta + j);
    }
    hipLaunchKernelGGL(tridiag_min_kernel, dim3(1), dim3(256), 0, st, sc->alpha, sc->beta, m, sc->y, &sc->eval);
    // the Ritz vector, normalised, becomes v_0 (and theta)
    hipLaunchKernelGGL(ritz_kernel, dim3(eb), dim3(256), 0, st, th, V, d.ld, m, sc->y, n);
    mdot(th, 1, th, sc->tmp, nullptr, 0, 0);
    hipLaunchKernelGGL(normalize_kernel, dim3(eb), dim3(256), 0, st, V, th, n, sc->tmp, nullptr, 0.0, nullptr);
    hipLaunchKernelGGL(normalize_kernel, dim3(eb), dim3(256), 0, st, th, th, n, sc->tmp, nullptr, 0.0, nullptr);
  }
  // residual |H theta - E theta| of the final vector
  TN_TRY(apply_h(V, w));
  hipLaunchKernelGGL(residual_kernel, dim3(eb), dim3(256), 0, st, w, V, &sc->eval, n);
  mdot(w, 1, w, sc->tmp, nullptr, 0, 0);
  hipLaunchKernelGGL(sqrt_to_kernel, dim3(1), dim3(1), 0, st, sc->tmp, &sc->resid);
  hipLaunchKernelGGL(energy_out_kernel, dim3(1), dim3(1), 0, st, sc, out2);
  return hip_check(hipGetLastError(), "dmrg eigensolve");
}

}  // extern "C"
