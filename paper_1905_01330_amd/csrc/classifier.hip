// MPS classifier of section IV.A on the GPU: forward scores, softmax
// cross-entropy, and the gradient with respect to every site tensor.
//
// Scores f[b, l] = <W^l, Phi(x_b)> with Phi(p) = (cos(pi p/2), sin(pi p/2))
// per pixel and one MPS whose centre site carries the label leg.  The left
// chain absorbs sites 0..c-1 into v (v_{k+1} = (v_k (x) Phi_k) . A_k) and
// the right chain absorbs sites N-1..c+1 into u (u_k = Phi_k . (A_k . u_{k+1})).
//
// Chain kernel: one workgroup owns 16 samples and walks a run of sites with
// the samples' vectors resident in LDS in FP64; each site is a 16-row FP64
// matrix-core product against the site tensor (FP32 in HBM, widened
// exactly), followed by an exact power-of-two rescale per sample (exponents
// kept as integers).  Up to four independent runs share one launch.  The
// forward stores a vector every `ckpt_every` sites; the backward recomputes
// each segment from its checkpoint while carrying the adjoint through it
// with the mirrored step, then forms the segment's weight gradients as one
// batched batch-reduction GEMM on the contraction kernel.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "internal.h"

namespace tn {

typedef float f32x4c_t __attribute__((ext_vector_type(4)));

constexpr int kRB = 16;        // samples per workgroup (rows of a 16x16 block)
constexpr int kMaxSeg = 64;    // sites per chain-kernel launch

struct ChainArgs {
  const float* w[kMaxSeg];  // site tensors of the run, in step order
  int first_site;         // site of step 0; step j is at first_site + dir * j
  int dir;
  int n_steps;
  int step_type;          // 0: v' = (v (x) Phi) . A   1: u' = Phi . (A . u)
  int n_sites;            // chain length (site 0 and n_sites-1 have a bond of 1)
  int chi;
  const float* pixels;    // [B, n_sites]
  int B;
  const float* v_in;      // vector block or NULL (unit vector, exponent 0)
  float* v_out;           // vector block (final vectors), may be NULL
  float* store;           // step inputs, may be NULL: step st's vectors at store + st * B * CHI,
  int64_t store_exp;      // its exponents at store + store_exp + st * B
  int lo;                 // v_in and v_out carry their low parts (see vblock_floats)
};

// A "vector block" holds B vectors of length CHI (zero beyond their bond
// dimension), then B exponents stored as floats, then the low parts of the
// B vectors: value = (hi + lo) * 2^e with hi = fl32(v), lo = fl32(v - hi).
// The running vectors handed from one chain launch to the next (and the
// checkpoints) keep the low parts, so the FP64 chain loses about 2^-48, not
// 2^-24, at every hand-off: random transfer matrices amplify a rounding of
// the running vector many times over by the end of the chain.  Blocks that
// only feed FP32 GEMM operands (adjoints, recomputed segment vectors) do
// not use the low parts.
__host__ __device__ inline int64_t vblock_floats(int B, int chi) { return 2 * (int64_t)B * chi + B; }
__host__ __device__ inline int64_t vblock_lo(int B, int chi) { return (int64_t)B * chi + B; }

typedef double f64x4_t __attribute__((ext_vector_type(4)));

// One run of sites for one chain.  The running vectors and the products are
// FP64 (FP64 matrix cores, v_mfma_f64_16x16x4): a 784-site chain of FP32
// steps would round the vector at every site, and those errors compound.
// Site tensors and pixels are read as FP32 and widened exactly.
// ---------------------------------------------------------------------------
// Chain kernel.  A workgroup owns 16 samples and has one wave per 16-wide
// block of output columns (CHI / 16 waves).  Per site it forms its block of
// the next vector with FP64 16x16x4 MFMAs, writes it to LDS unnormalised
// together with the block's row maxima, and meets the other waves at one
// barrier; every wave then derives each row's power-of-two normaliser from
// the maxima and applies it while reading the vector in the next site.  For
// CHI <= 128 the site tensor of the next site is loaded into registers
// while the current site's MFMAs run (two register sets, sites unrolled by
// two); CHI = 256 loads its tensor in chunks within the site.
template <int CHI>
struct ChainSmem {
  static constexpr int NW = CHI / 16;
  double vec[2][kRB][CHI + 2];
  double phi[kMaxSeg][kRB][2];
  double pmax[2][NW][kRB];
  const float* w[kMaxSeg];
  int din[kMaxSeg], dout[kMaxSeg];
};

template <int CHI, int TYPE>
struct ChainRegs {
  // site-tensor registers of one site for the lane's column block
  static constexpr bool PREFETCH = CHI <= 128;
  static constexpr int KI0 = CHI / 2;        // type 0: MFMA steps (k = 2a + s in groups of 4)
  static constexpr int NV1 = CHI / 16;       // type 1: float4 per row slice (z in groups of 4 per lane)
  float w0[TYPE == 0 && PREFETCH ? KI0 : 1];
  f32x4c_t wa[TYPE == 1 && PREFETCH ? NV1 : 1], wb[TYPE == 1 && PREFETCH ? NV1 : 1];
};

template <int CHI, int TYPE>
__device__ __forceinline__ void chain_load(ChainRegs<CHI, TYPE>& R, const float* W, int col, int g) {
  if constexpr (ChainRegs<CHI, TYPE>::PREFETCH) {
    if constexpr (TYPE == 0) {
#pragma unroll
      for (int kk = 0; kk < CHI / 2; ++kk) R.w0[kk] = W[(int64_t)(4 * kk + g) * CHI + col];
    } else {
      const float* r0 = W + ((int64_t)col * 2) * CHI + g * (CHI / 4);
#pragma unroll
      for (int j = 0; j < CHI / 16; ++j) {
        R.wa[j] = *reinterpret_cast<const f32x4c_t*>(r0 + 4 * j);
        R.wb[j] = *reinterpret_cast<const f32x4c_t*>(r0 + CHI + 4 * j);
      }
    }
  }
}

template <int CHI, int TYPE, int SET>
__device__ __forceinline__ void chain_step(const ChainArgs& a, ChainSmem<CHI>& sm, ChainRegs<CHI, TYPE> (&regs)[2],
                                           int st, int& cur, double& scl, int& ex, int b0) {
  constexpr int NW = CHI / 16;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int row = lane & 15, g = lane >> 4;
  const int col = wave * 16 + row;          // this lane's output column (type 0: z, type 1: a)
  const int din = sm.din[st], dout = sm.dout[st];
  const float* W = sm.w[st];
  const bool fast = din == CHI && dout == CHI && (TYPE == 0 || (reinterpret_cast<uintptr_t>(W) & 15) == 0);
  const int nxt = cur ^ 1, par = st & 1;
  // prefetch the next site's tensor into the other register set
  if constexpr (ChainRegs<CHI, TYPE>::PREFETCH) {
    if (st + 1 < a.n_steps) {
      const float* Wn = sm.w[st + 1];
      if (sm.din[st + 1] == CHI && sm.dout[st + 1] == CHI &&
          (TYPE == 0 || (reinterpret_cast<uintptr_t>(Wn) & 15) == 0))
        chain_load<CHI, TYPE>(regs[SET ^ 1], Wn, col, g);
    }
  }
  f64x4_t acc0 = {0.0, 0.0, 0.0, 0.0}, acc1 = acc0;
  if (TYPE == 0) {
    // out[r, z] = sum_{a, s} x[r, a] phi[r, s] W[(a s), z]   (k = 2a + s)
    const double p0 = sm.phi[st][row][0] * scl, p1 = sm.phi[st][row][1] * scl;
    if (fast && ChainRegs<CHI, TYPE>::PREFETCH) {
#pragma unroll
      for (int kk = 0; kk < CHI / 2; ++kk) {
        const int k = 4 * kk + g;
        const double xv = sm.vec[cur][row][k >> 1] * ((k & 1) ? p1 : p0);
        acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(xv, (double)regs[SET].w0[kk], acc0, 0, 0, 0);
      }
    } else if (fast) {
      constexpr int CH = 16;
      for (int k0 = 0; k0 < CHI / 2; k0 += CH) {
        float wv[CH];
#pragma unroll
        for (int q = 0; q < CH; ++q) wv[q] = W[(int64_t)(4 * (k0 + q) + g) * CHI + col];
#pragma unroll
        for (int q = 0; q < CH; ++q) {
          const int k = 4 * (k0 + q) + g;
          const double xv = sm.vec[cur][row][k >> 1] * ((k & 1) ? p1 : p0);
          acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(xv, (double)wv[q], acc0, 0, 0, 0);
        }
      }
    } else if (col - row < dout) {
      const int K4 = (2 * din + 3) >> 2;
      for (int kk = 0; kk < K4; ++kk) {
        const int k = 4 * kk + g, aa = k >> 1;
        double xv = 0.0, wv = 0.0;
        if (aa < din) {
          xv = sm.vec[cur][row][aa] * ((k & 1) ? p1 : p0);
          if (col < dout) wv = (double)W[(int64_t)k * dout + col];
        }
        acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(xv, wv, acc0, 0, 0, 0);
      }
    }
  } else {
    // out[r, a] = sum_s phi[r, s] sum_z x[r, z] W[a, s, z]
    if (fast && ChainRegs<CHI, TYPE>::PREFETCH) {
      constexpr int KI = CHI / 4;
#pragma unroll
      for (int kk = 0; kk < KI; ++kk) {
        const double xv = sm.vec[cur][row][g * KI + kk] * scl;
        acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(xv, (double)regs[SET].wa[kk >> 2][kk & 3], acc0, 0, 0, 0);
        acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(xv, (double)regs[SET].wb[kk >> 2][kk & 3], acc1, 0, 0, 0);
      }
    } else if (fast) {
      constexpr int KI = CHI / 4;
      const float* r0 = W + ((int64_t)col * 2) * CHI + g * KI;
      constexpr int CH = 4;    // float4 per chunk (16 z values of the lane's slice)
      for (int j0 = 0; j0 < KI / 4; j0 += CH) {
        f32x4c_t wa[CH], wb[CH];
#pragma unroll
        for (int j = 0; j < CH; ++j) {
          wa[j] = *reinterpret_cast<const f32x4c_t*>(r0 + 4 * (j0 + j));
          wb[j] = *reinterpret_cast<const f32x4c_t*>(r0 + CHI + 4 * (j0 + j));
        }
#pragma unroll
        for (int kk = 0; kk < 4 * CH; ++kk) {
          const double xv = sm.vec[cur][row][g * KI + 4 * j0 + kk] * scl;
          acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(xv, (double)wa[kk >> 2][kk & 3], acc0, 0, 0, 0);
          acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(xv, (double)wb[kk >> 2][kk & 3], acc1, 0, 0, 0);
        }
      }
    } else if (col - row < dout) {
      const int K4 = (din + 3) >> 2;
      for (int kk = 0; kk < K4; ++kk) {
        const int z = 4 * kk + g;
        double xv = 0.0, w0 = 0.0, w1 = 0.0;
        if (z < din) {
          xv = sm.vec[cur][row][z] * scl;
          if (col < dout) {
            w0 = (double)W[((int64_t)col * 2 + 0) * din + z];
            w1 = (double)W[((int64_t)col * 2 + 1) * din + z];
          }
        }
        acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(xv, w0, acc0, 0, 0, 0);
        acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(xv, w1, acc1, 0, 0, 0);
      }
    }
  }
  // FP64 16x16x4 result: lane (col + 16 g) register r holds row 4 r + g
  double outv[4];
  double m[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int rr = r * 4 + g;
    double v = TYPE == 0 ? acc0[r] : sm.phi[st][rr][0] * acc0[r] + sm.phi[st][rr][1] * acc1[r];
    if (col >= dout) v = 0.0;
    outv[r] = v;
    sm.vec[nxt][rr][col] = v;
    m[r] = fabs(v);
  }
#pragma unroll
  for (int o = 8; o >= 1; o >>= 1)
#pragma unroll
    for (int r = 0; r < 4; ++r) m[r] = fmax(m[r], __shfl_xor(m[r], o, 16));
  if (row == 0) {
#pragma unroll
    for (int r = 0; r < 4; ++r) sm.pmax[par][wave][r * 4 + g] = m[r];
  }
  __syncthreads();
  // the row normaliser 2^-e (e the binary exponent of the row maximum)
  auto row_exp = [&](int rr) {
    double mm = 0.0;
#pragma unroll
    for (int w = 0; w < NW; ++w) mm = fmax(mm, sm.pmax[par][w][rr]);
    return (mm > 0.0 && mm < 1e300) ? ilogb(mm) : 0;
  };
  const int e = row_exp(row);
  // a stored block holds this site's output (the next site's input), normalised
  float* dst = nullptr;     // vectors of the block to write
  float* dste = nullptr;    // its exponents
  float* dstl = nullptr;    // its low parts (running-vector hand-off only)
  if (a.store && st + 1 < a.n_steps) {
    dst = a.store + (int64_t)(st + 1) * a.B * CHI;
    dste = a.store + a.store_exp + (int64_t)(st + 1) * a.B;
  } else if (a.v_out && st + 1 == a.n_steps) {
    dst = a.v_out;
    dste = a.v_out + (int64_t)a.B * CHI;
    if (a.lo) dstl = a.v_out + vblock_lo(a.B, CHI);
  }
  if (dst) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int rr = r * 4 + g, b = b0 + rr;
      const int er = row_exp(rr);
      if (b < a.B) {
        const double x = ldexp(outv[r], -er);
        const float hi = (float)x;
        dst[(int64_t)b * CHI + col] = hi;
        if (dstl) dstl[(int64_t)b * CHI + col] = (float)(x - (double)hi);
      }
    }
    if (wave == 0 && g == 0 && b0 + row < a.B) dste[b0 + row] = (float)(ex + e);
  }
  ex += e;
  scl = ldexp(1.0, -e);
  cur = nxt;
}

template <int CHI, int TYPE>
__device__ __forceinline__ void chain_run(const ChainArgs& a, ChainSmem<CHI>& sm) {
  constexpr int NT = CHI / 16 * 64;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int row = lane & 15, g = lane >> 4;
  const int b0 = blockIdx.x * kRB;
  if (b0 >= a.B) return;
  if (tid == 0) {
#pragma unroll
    for (int j = 0; j < kMaxSeg; ++j)
      if (j < a.n_steps) {
        const int k = a.first_site + a.dir * j;
        const int dl = k == 0 ? 1 : a.chi, dr = k == a.n_sites - 1 ? 1 : a.chi;
        sm.w[j] = a.w[j];
        sm.din[j] = TYPE == 0 ? dl : dr;
        sm.dout[j] = TYPE == 0 ? dr : dl;
      }
  }
  // feature map of every site of the run
  for (int e = tid; e < a.n_steps * kRB * 2; e += NT) {
    const int st = e / (2 * kRB), r = (e >> 1) % kRB, sc = e & 1, b = b0 + r;
    const int k = a.first_site + a.dir * st;
    const double p = b < a.B ? (double)a.pixels[(int64_t)b * a.n_sites + k] : 0.0;
    double sv, cv;
    sincospi(0.5 * p, &sv, &cv);
    sm.phi[st][r][sc] = sc == 0 ? cv : sv;
  }
  for (int e = tid; e < kRB * CHI; e += NT) {
    const int r = e / CHI, i = e % CHI, b = b0 + r;
    double x = 0.0;
    if (b < a.B) {
      if (a.v_in) {
        x = (double)a.v_in[(int64_t)b * CHI + i];
        if (a.lo) x += (double)a.v_in[vblock_lo(a.B, CHI) + (int64_t)b * CHI + i];
      } else {
        x = i == 0 ? 1.0 : 0.0;
      }
    }
    sm.vec[0][r][i] = x;
  }
  int ex = (a.v_in && b0 + row < a.B) ? (int)a.v_in[(int64_t)a.B * CHI + b0 + row] : 0;
  double scl = 1.0;
  // the first site's input, stored as given
  if (a.store) {
    const int col = wave * 16 + row;
    for (int r = g; r < kRB; r += 4) {
      const int b = b0 + r;
      if (b < a.B) {
        const double x = a.v_in ? (double)a.v_in[(int64_t)b * CHI + col] : (col == 0 ? 1.0 : 0.0);
        a.store[(int64_t)b * CHI + col] = (float)x;
      }
    }
    if (wave == 0 && g == 0 && b0 + row < a.B) a.store[a.store_exp + b0 + row] = (float)ex;
  }
  ChainRegs<CHI, TYPE> regs[2];
  __syncthreads();
  if constexpr (ChainRegs<CHI, TYPE>::PREFETCH) {
    if (sm.din[0] == CHI && sm.dout[0] == CHI && (TYPE == 0 || (reinterpret_cast<uintptr_t>(sm.w[0]) & 15) == 0))
      chain_load<CHI, TYPE>(regs[0], sm.w[0], wave * 16 + row, g);
  }
  int cur = 0;
  for (int st = 0; st < a.n_steps; st += 2) {
    chain_step<CHI, TYPE, 0>(a, sm, regs, st, cur, scl, ex, b0);
    if (st + 1 < a.n_steps) chain_step<CHI, TYPE, 1>(a, sm, regs, st + 1, cur, scl, ex, b0);
  }
  // a run of zero sites (never launched) would leave v_out unwritten
}

// blockIdx.y selects one of up to four independent runs (left and right
// chains, recomputation and adjoint) advancing in one launch
template <int CHI>
__global__ void __launch_bounds__(CHI / 16 * 64)
    chain_kernel(const ChainArgs a0, const ChainArgs a1, const ChainArgs a2, const ChainArgs a3) {
  __shared__ ChainSmem<CHI> sm;
  switch (blockIdx.y) {
    case 0:
      if (a0.step_type == 0) chain_run<CHI, 0>(a0, sm); else chain_run<CHI, 1>(a0, sm);
      break;
    case 1:
      if (a1.step_type == 0) chain_run<CHI, 0>(a1, sm); else chain_run<CHI, 1>(a1, sm);
      break;
    case 2:
      if (a2.step_type == 0) chain_run<CHI, 0>(a2, sm); else chain_run<CHI, 1>(a2, sm);
      break;
    default:
      if (a3.step_type == 0) chain_run<CHI, 0>(a3, sm); else chain_run<CHI, 1>(a3, sm);
      break;
  }
}

// X[b, a, s] = v[b, a] * Phi_s(x_{b, site}) * (with_scale ? 2^(e_v[b] + e_w[b]) : 1)
__global__ void expand_kernel(const float* vblk, const float* wblk_exp, const float* pixels, int n_pix, int site, int B,
                              int chi, int d, float* x) {
  const int64_t total = (int64_t)B * d * 2;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int s = (int)(e & 1);
    const int64_t ba = e >> 1;
    const int b = (int)(ba / d), aa = (int)(ba % d);
    float sv, cv;
    sincospif(0.5f * pixels[(int64_t)b * n_pix + site], &sv, &cv);
    float val = vblk[(int64_t)b * chi + aa] * (s == 0 ? cv : sv);
    if (wblk_exp) {
      const int ex = (int)vblk[(int64_t)B * chi + b] + (int)wblk_exp[b];
      val = ldexpf(val, ex);
    }
    x[e] = val;
  }
}

// One segment of gradient operands at once.  A segment buffer holds E
// vector slots of B x pc floats followed by E x B exponents (at + eoff).
// Batch entry j is site k_j = k0 - j:
//   X_j[b, a, s] = V_j[b, a] Phi_s(x_{b, k_j}) 2^(e_V(b) + e_G(b))
// with V_j in slot n-1-j of vsrc and e_G the exponents of slot j of gsrc
// (the GEMM's other operand).  a runs over chi.
__global__ void expand_seg_kernel(const float* vsrc, const float* gsrc, int64_t eoff, int n, int k0,
                                  const float* pixels, int n_pix, int B, int pc, int chi, float* x) {
  const int j = blockIdx.y;
  const float* v = vsrc + (int64_t)(n - 1 - j) * B * pc;
  const float* ve = vsrc + eoff + (int64_t)(n - 1 - j) * B;
  const float* ge = gsrc + eoff + (int64_t)j * B;
  const int k = k0 - j;
  float* xj = x + (int64_t)j * B * chi * 2;
  const int64_t total = (int64_t)B * chi * 2;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int s = (int)(e & 1);
    const int64_t ba = e >> 1;
    const int b = (int)(ba / chi), aa = (int)(ba % chi);
    float sv, cv;
    sincospif(0.5f * pixels[(int64_t)b * n_pix + k], &sv, &cv);
    const int ex = (int)ve[b] + (int)ge[b];
    xj[e] = ldexpf(v[(int64_t)b * pc + aa] * (s == 0 ? cv : sv), ex);
  }
}

struct ScatterArgs {
  float* dst[kMaxSeg];
  int64_t st[kMaxSeg][3];
};

// dA_{k_j}[a, s, z] = sum_c G_{j,c}[a, s, z] (the S batch chunks, summed in
// a fixed order) for a < d_left(k_j), z < d_right(k_j)
__global__ void scatter_grad_kernel(const float* gbuf, int n, int S, int k0, int n_sites, int chi, const ScatterArgs sa) {
  const int j = blockIdx.y;
  const int k = k0 - j;
  const int dl = k == 0 ? 1 : chi, dr = k == n_sites - 1 ? 1 : chi;
  const int64_t blk = (int64_t)chi * 2 * chi;
  const float* src = gbuf + (int64_t)j * S * blk;
  float* dst = nullptr;
  int64_t s0 = 0, s1 = 0, s2 = 0;
#pragma unroll
  for (int q = 0; q < kMaxSeg; ++q)
    if (q == j) {
      dst = sa.dst[q];
      s0 = sa.st[q][0];
      s1 = sa.st[q][1];
      s2 = sa.st[q][2];
    }
  const int64_t total = (int64_t)dl * 2 * dr;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int z = (int)(e % dr);
    const int64_t as = e / dr;
    const int sidx = (int)(as & 1), aa = (int)(as >> 1);
    const int64_t o = ((int64_t)aa * 2 + sidx) * chi + z;
    float v = 0.f;
    for (int c = 0; c < S; ++c) v += src[c * blk + o];
    dst[aa * s0 + sidx * s1 + z * s2] = v;
  }
}

// logits[b, l] = 2^(e_v + e_u) sum_z T[b, l, z] u[b, z]
__global__ void logits_kernel(const float* t, const float* ublk, const float* vblk, int B, int L, int chi, int du,
                              float* logits, int64_t ls0, int64_t ls1) {
  const int64_t total = (int64_t)B * L;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int b = (int)(e / L), l = (int)(e % L);
    double acc = 0.0;
    for (int z = 0; z < du; ++z) acc += (double)t[((int64_t)b * L + l) * du + z] * (double)ublk[(int64_t)b * chi + z];
    const int ex = (int)vblk[(int64_t)B * chi + b] + (int)ublk[(int64_t)B * chi + b];
    logits[b * ls0 + l * ls1] = (float)ldexp(acc, ex);
  }
}

// gu[b, l, z] = g[b, l] * u[b, z] * 2^scale_exp(b)   (scale_exp from up to two exponent blocks)
__global__ void gu_kernel(const float* g, int64_t gs0, int64_t gs1, const float* ublk, const float* e1blk, int B, int L,
                          int chi, int du, float* gu) {
  const int64_t total = (int64_t)B * L * du;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int z = (int)(e % du);
    const int64_t bl = e / du;
    const int b = (int)(bl / L), l = (int)(bl % L);
    float v = g[b * gs0 + l * gs1] * ublk[(int64_t)b * chi + z];
    if (e1blk) v = ldexpf(v, (int)e1blk[(int64_t)B * chi + b] + (int)ublk[(int64_t)B * chi + b]);
    gu[e] = v;
  }
}

// abar[b, a] = sum_s Phi_s(x_c) Y[b, a, s]  into a vector block with exponent taken from `expblk`
__global__ void phi_contract_kernel(const float* y, const float* pixels, int n_pix, int site, int B, int d, int chi,
                                    const float* expblk, float* out) {
  const int64_t total = (int64_t)B * chi;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int b = (int)(e / chi), aa = (int)(e % chi);
    float v = 0.f;
    if (aa < d) {
      float sv, cv;
      sincospif(0.5f * pixels[(int64_t)b * n_pix + site], &sv, &cv);
      v = cv * y[((int64_t)b * d + aa) * 2 + 0] + sv * y[((int64_t)b * d + aa) * 2 + 1];
    }
    out[e] = v;
    if (aa == 0) out[(int64_t)B * chi + b] = expblk[(int64_t)B * chi + b];
  }
}

// ubar[b, z] = sum_l g[b, l] T[b, l, z]  into a vector block with exponent from `expblk`
__global__ void gt_kernel(const float* g, int64_t gs0, int64_t gs1, const float* t, int B, int L, int du, int chi,
                          const float* expblk, float* out) {
  const int64_t total = (int64_t)B * chi;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int b = (int)(e / chi), z = (int)(e % chi);
    float v = 0.f;
    if (z < du) {
      double acc = 0.0;
      for (int l = 0; l < L; ++l) acc += (double)g[b * gs0 + l * gs1] * (double)t[((int64_t)b * L + l) * du + z];
      v = (float)acc;
    }
    out[e] = v;
    if (z == 0) out[(int64_t)B * chi + b] = expblk[(int64_t)B * chi + b];
  }
}

__global__ void softmax_xent_kernel(const float* logits, int64_t ls0, int64_t ls1, const int64_t* labels, int B, int L,
                                    double* loss_part, float* dlogits, int64_t ds0, int64_t ds1) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B) return;
  double m = -1e300;
  for (int l = 0; l < L; ++l) m = fmax(m, (double)logits[b * ls0 + l * ls1]);
  double z = 0.0;
  for (int l = 0; l < L; ++l) z += exp((double)logits[b * ls0 + l * ls1] - m);
  const int64_t yl = labels[b];
  if (yl < 0 || yl >= L) {  // a label outside 0..L-1 has no loss: NaN marks it
    loss_part[b] = __longlong_as_double(0x7ff8000000000000ll);
    for (int l = 0; l < L; ++l) dlogits[b * ds0 + l * ds1] = __int_as_float(0x7fc00000);
    return;
  }
  const int y = (int)yl;
  loss_part[b] = m + log(z) - (double)logits[b * ls0 + y * ls1];
  for (int l = 0; l < L; ++l) {
    const double p = exp((double)logits[b * ls0 + l * ls1] - m) / z;
    dlogits[b * ds0 + l * ds1] = (float)((p - (l == y ? 1.0 : 0.0)) / B);
  }
}

__global__ void mean_kernel(const double* part, int n, double* out) {
  __shared__ double red[4];
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) s += part[i];
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) s += __shfl_xor(s, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) out[0] = (red[0] + red[1] + red[2] + red[3]) / n;
}

static unsigned blocks_of(int64_t n) { return (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 16384)); }

// ---------------------------------------------------------------------------
// host side

namespace {

struct Geometry {
  int N, c, L, B, chi, E;
  int pad_chi;                 // chain-kernel CHI (16, 32, 64, 128, 256)
  std::vector<int> left_b;     // left segment boundaries 0 = s_0 < ... < s_m = c
  std::vector<int> right_b;    // right boundaries N = t_0 > ... > t_m = c + 1
  int64_t vb;                  // floats per vector block
  size_t ckpt_floats;
  int S;                       // batch chunks of the weight-gradient GEMMs
};

// Batch chunks for the weight-gradient GEMMs (K = batch is long, the output
// 2 chi x chi small): split the batch while it divides evenly, the chunks
// keep at least 64 samples and a segment has fewer than 2048 64 x 64 tiles.
int grad_chunks(int B, int chi, int E) {
  const int64_t tiles = (int64_t)((2 * chi + 63) / 64) * ((chi + 63) / 64);
  int S = 1;
  while (S < 16 && B % (2 * S) == 0 && B / (2 * S) >= 64 && (int64_t)E * S * tiles < 2048) S *= 2;
  return S;
}

int pad_of(int chi) {
  for (int p : {16, 32, 64, 128, 256})
    if (chi <= p) return p;
  return -1;
}

int32_t geometry(int32_t N, int32_t c, int32_t L, int32_t B, int32_t chi, int32_t E, Geometry& g) {
  if (N < 3 || c < 1 || c > N - 2) return fail(TN_ERR_INVALID_ARGUMENT, "need n_sites >= 3 and 1 <= label_site <= n_sites - 2");
  if (L < 1 || B < 1 || chi < 1) return fail(TN_ERR_INVALID_ARGUMENT, "n_labels, batch and chi must be >= 1");
  if (E < 1 || E > kMaxSeg) return fail(TN_ERR_INVALID_ARGUMENT, "ckpt_every must be in 1..%d", kMaxSeg);
  g.N = N;
  g.c = c;
  g.L = L;
  g.B = B;
  g.chi = chi;
  g.E = E;
  g.pad_chi = pad_of(chi);
  if (g.pad_chi < 0) return fail(TN_ERR_UNSUPPORTED, "bond dimension above 256");
  g.left_b.clear();
  for (int s = 0; s < c; s += E) g.left_b.push_back(s);
  g.left_b.push_back(c);
  g.right_b.clear();
  for (int t = N; t > c + 1; t -= E) g.right_b.push_back(t);
  g.right_b.push_back(c + 1);
  g.vb = vblock_floats(B, g.pad_chi);
  g.S = grad_chunks(B, chi, E);
  g.ckpt_floats = (size_t)(g.left_b.size() + g.right_b.size()) * g.vb;
  return TN_OK;
}

size_t al(size_t x) { return (x + 255) & ~(size_t)255; }

struct WsLayout {
  size_t vtmp0, vtmp1, xbuf, tbuf, ybuf, gubuf, seg_v[2], seg_g[2], xseg[2], gbuf[2], part, total;
};

// per chain side (left, right): recomputed vectors, adjoints, expanded
// gradient operands and dense gradient blocks of one segment
WsLayout ws_layout(const Geometry& g) {
  WsLayout w;
  const size_t vb = (size_t)g.vb * 4;
  const size_t E = g.E;
  size_t o = 0;
  w.vtmp0 = o; o += al(vb);
  w.vtmp1 = o; o += al(vb);
  w.xbuf = o; o += al((size_t)g.B * g.chi * 2 * 4);
  w.tbuf = o; o += al((size_t)g.B * g.L * g.chi * 4);
  w.ybuf = o; o += al((size_t)g.B * g.chi * 2 * 4);
  w.gubuf = o; o += al((size_t)g.B * g.L * g.chi * 4);
  for (int side = 0; side < 2; ++side) {
    w.seg_v[side] = o; o += al(E * vb);
    w.seg_g[side] = o; o += al(E * vb);
    w.xseg[side] = o; o += al(E * (size_t)g.B * g.chi * 2 * 4);
    w.gbuf[side] = o; o += al(E * (size_t)g.S * g.chi * 2 * g.chi * 4);
  }
  w.part = o; o += al((size_t)g.B * 8);
  w.total = o;
  return w;
}

int32_t check_sites(const Geometry& g, const tn_tensor* sites, const char* name) {
  if (!sites) return fail(TN_ERR_INVALID_ARGUMENT, "%s is NULL", name);
  for (int k = 0; k < g.N; ++k) {
    char nm[48];
    snprintf(nm, sizeof(nm), "%s[%d]", name, k);
    TN_TRY(check_tensor(&sites[k], nm, TN_F32));
    const tn_tensor& t = sites[k];
    const int64_t dl = k == 0 ? 1 : g.chi, dr = k == g.N - 1 ? 1 : g.chi;
    if (k == g.c) {
      if (t.rank != 4 || t.shape[0] != dl || t.shape[1] != 2 || t.shape[2] != g.L || t.shape[3] != dr)
        return fail(TN_ERR_SHAPE_MISMATCH, "%s must be [%lld, 2, %d, %lld]", nm, (long long)dl, g.L, (long long)dr);
    } else if (t.rank != 3 || t.shape[0] != dl || t.shape[1] != 2 || t.shape[2] != dr) {
      return fail(TN_ERR_SHAPE_MISMATCH, "%s must be [%lld, 2, %lld]", nm, (long long)dl, (long long)dr);
    }
    int64_t st = 1;
    for (int q = t.rank - 1; q >= 0; --q) {
      if (t.stride[q] != st) return fail(TN_ERR_UNSUPPORTED, "%s must be contiguous", nm);
      st *= t.shape[q];
    }
  }
  return TN_OK;
}

ChainArgs chain_args(const Geometry& g, const tn_tensor* sites, const float* pixels, int step_type, int first_site,
                     int dir, int n_steps, const float* v_in, float* v_out, float* store, int lo) {
  ChainArgs a;
  std::memset(&a, 0, sizeof(a));
  a.first_site = first_site;
  a.dir = dir;
  a.n_steps = n_steps;
  a.step_type = step_type;
  a.n_sites = g.N;
  a.chi = g.chi;
  a.pixels = pixels;
  a.B = g.B;
  a.v_in = v_in;
  a.v_out = v_out;
  a.store = store;
  a.lo = lo;
  a.store_exp = (int64_t)g.E * g.B * g.pad_chi;   // segment buffers: E vector slots, then E x B exponents
  for (int j = 0; j < n_steps; ++j) a.w[j] = static_cast<const float*>(sites[first_site + dir * j].data);
  return a;
}

// up to four independent runs in one launch
int32_t launch_chains(const Geometry& g, const std::vector<ChainArgs>& runs, hipStream_t st) {
  std::vector<ChainArgs> r;
  for (const ChainArgs& a : runs)
    if (a.n_steps > 0) r.push_back(a);
  if (r.empty()) return TN_OK;
  if (r.size() > 4) return fail(TN_ERR_INVALID_ARGUMENT, "at most four chain runs per launch");
  const dim3 grid((unsigned)((g.B + kRB - 1) / kRB), (unsigned)r.size());
  while (r.size() < 4) r.push_back(r[0]);
  // one wave per 16 output columns
  switch (g.pad_chi) {
    case 16: hipLaunchKernelGGL(chain_kernel<16>, grid, dim3(64), 0, st, r[0], r[1], r[2], r[3]); break;
    case 32: hipLaunchKernelGGL(chain_kernel<32>, grid, dim3(128), 0, st, r[0], r[1], r[2], r[3]); break;
    case 64: hipLaunchKernelGGL(chain_kernel<64>, grid, dim3(256), 0, st, r[0], r[1], r[2], r[3]); break;
    case 128: hipLaunchKernelGGL(chain_kernel<128>, grid, dim3(512), 0, st, r[0], r[1], r[2], r[3]); break;
    default: hipLaunchKernelGGL(chain_kernel<256>, grid, dim3(1024), 0, st, r[0], r[1], r[2], r[3]); break;
  }
  return hip_check(hipGetLastError(), "chain kernel");
}

int32_t launch_chain(const Geometry& g, const tn_tensor* sites, const float* pixels, int step_type, int first_site,
                     int dir, int n_steps, const float* v_in, float* v_out, float* store, int lo, hipStream_t st) {
  if (n_steps <= 0) return TN_OK;
  return launch_chains(g, {chain_args(g, sites, pixels, step_type, first_site, dir, n_steps, v_in, v_out, store, lo)},
                       st);
}

// Weight gradients of one segment: dA_{k_j} = sum_b X_j[b, (a s)] G_j[b, z]
// for j < n, k_j = k0 - j, X_j formed from vsrc (see expand_seg_kernel) and
// G_j the vectors of slot j of gsrc.  One batched GEMM over (j, chunk c of
// the batch) into S partial blocks per site, then a scatter that sums them
// into the caller's gradient tensors.
int32_t segment_grads(const Geometry& g, const float* vsrc, const float* gsrc, int n, int k0, const float* px,
                      float* xseg, float* gbuf, tn_tensor* dsites, int32_t prec, hipStream_t st) {
  if (n <= 0) return TN_OK;
  const int B = g.B, chi = g.chi, pc = g.pad_chi, S = g.S, Bc = B / S;
  const int64_t eoff = (int64_t)g.E * B * pc;
  hipLaunchKernelGGL(expand_seg_kernel, dim3(std::min<unsigned>(blocks_of((int64_t)B * chi * 2), 2048), n), dim3(256),
                     0, st, vsrc, gsrc, eoff, n, k0, px, g.N, B, pc, chi, xseg);
  TN_TRY(hip_check(hipGetLastError(), "expand segment"));
  tn_tensor xv = make_view(xseg, TN_F32, {Bc, chi, 2});
  tn_tensor gv;
  std::memset(&gv, 0, sizeof(gv));
  gv.data = const_cast<float*>(gsrc);
  gv.dtype = TN_F32;
  gv.rank = 2;
  gv.shape[0] = Bc;
  gv.shape[1] = chi;
  gv.stride[0] = pc;
  gv.stride[1] = 1;
  tn_tensor ov = make_view(gbuf, TN_F32, {chi, 2, chi});
  const int32_t pa[1] = {0}, pb[1] = {0};
  GemmDesc d;
  TN_TRY(plan_gemm(xv, gv, 1, pa, pb, ov, d));
  // batch entry j * S + c: X_j rows and G_j rows of chunk c, partial block (j, c)
  d.batch = n * S;
  d.a_bs = (int64_t)Bc * chi * 2;
  d.b_bs = (int64_t)Bc * pc;
  d.c_bs = (int64_t)chi * 2 * chi;
  choose_modes(d);
  TN_TRY(launch_gemm(d, prec, st));
  ScatterArgs sa;
  std::memset(&sa, 0, sizeof(sa));
  for (int j = 0; j < n; ++j) {
    const tn_tensor& t = dsites[k0 - j];
    sa.dst[j] = static_cast<float*>(t.data);
    for (int q = 0; q < 3; ++q) sa.st[j][q] = t.stride[q];
  }
  hipLaunchKernelGGL(scatter_grad_kernel, dim3(blocks_of((int64_t)chi * 2 * chi), n), dim3(256), 0, st, gbuf, n, S, k0,
                     g.N, chi, sa);
  return hip_check(hipGetLastError(), "scatter gradients");
}

// T[b, l, z] = sum_{a s} Xc[b, a, s] A_c[a, s, l, z]
int32_t label_t(const Geometry& g, const tn_tensor& ac, const float* x, float* t, int32_t prec, hipStream_t st) {
  tn_tensor xv = make_view(const_cast<float*>(x), TN_F32, {g.B, g.chi, 2});
  tn_tensor tv = make_view(t, TN_F32, {g.B, g.L, g.chi});
  const int32_t pa[2] = {1, 2}, pb[2] = {0, 1};
  return contract_between_impl(&xv, &ac, 2, pa, pb, &tv, nullptr, 0, prec, st);
}

// cumulative left/right forward: fills checkpoints, returns v_c and u_{c+1} blocks
int32_t forward_core(const Geometry& g, const tn_tensor* sites, const float* pixels, float* ckpt, hipStream_t st) {
  const size_t nl = g.left_b.size() - 1, nr = g.right_b.size() - 1, off = g.left_b.size();
  for (size_t j = 0; j < std::max(nl, nr); ++j) {
    std::vector<ChainArgs> runs;
    if (j < nl)  // slot 0 of each chain (the unit vector) is implicit
      runs.push_back(chain_args(g, sites, pixels, 0, g.left_b[j], 1, g.left_b[j + 1] - g.left_b[j],
                                j == 0 ? nullptr : ckpt + j * g.vb, ckpt + (j + 1) * g.vb, nullptr, 1));
    if (j < nr)
      runs.push_back(chain_args(g, sites, pixels, 1, g.right_b[j] - 1, -1, g.right_b[j] - g.right_b[j + 1],
                                j == 0 ? nullptr : ckpt + (off + j) * g.vb, ckpt + (off + j + 1) * g.vb, nullptr, 1));
    TN_TRY(launch_chains(g, runs, st));
  }
  return TN_OK;
}

__global__ void unit_block_kernel(float* blk, int B, int chi) {
  const int64_t total = vblock_floats(B, chi);
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x)
    blk[e] = (e < (int64_t)B * chi && e % chi == 0) ? 1.f : 0.f;
}

}  // namespace

}  // namespace tn

using namespace tn;

extern "C" {

int32_t tn_mps_classifier_ckpt_shape(int32_t n_sites, int32_t label_site, int32_t batch, int32_t chi,
                                     int32_t ckpt_every, int64_t* n_floats) {
  if (!n_floats) return fail(TN_ERR_INVALID_ARGUMENT, "n_floats is NULL");
  Geometry g;
  TN_TRY(geometry(n_sites, label_site, 1, batch, chi, ckpt_every, g));
  *n_floats = (int64_t)g.ckpt_floats;
  return TN_OK;
}

int32_t tn_mps_classifier_workspace(int32_t n_sites, int32_t label_site, int32_t n_labels, int32_t batch, int32_t chi,
                                    int32_t ckpt_every, size_t* bytes) {
  if (!bytes) return fail(TN_ERR_INVALID_ARGUMENT, "bytes is NULL");
  Geometry g;
  TN_TRY(geometry(n_sites, label_site, n_labels, batch, chi, ckpt_every, g));
  *bytes = ws_layout(g).total;
  return TN_OK;
}

int32_t tn_mps_classifier_forward(int32_t n_sites, int32_t label_site, int32_t n_labels, const tn_tensor* sites,
                                  const tn_tensor* pixels, tn_tensor* logits, float* ckpt, int32_t ckpt_every,
                                  void* workspace, size_t ws_bytes, int32_t prec, void* stream) {
  TN_TRY(check_tensor(pixels, "pixels", TN_F32));
  TN_TRY(check_tensor(logits, "logits", TN_F32));
  if (pixels->rank != 2 || pixels->shape[1] != n_sites || pixels->stride[1] != 1 || pixels->stride[0] != n_sites)
    return fail(TN_ERR_SHAPE_MISMATCH, "pixels must be a contiguous [B, n_sites] tensor");
  const int B = (int)pixels->shape[0];
  if (n_sites < 3 || !sites) return fail(TN_ERR_INVALID_ARGUMENT, "need n_sites >= 3 and sites");
  const int chi = (int)sites[1].shape[0];
  Geometry g;
  TN_TRY(geometry(n_sites, label_site, n_labels, B, chi, ckpt_every > 0 ? ckpt_every : 28, g));
  TN_TRY(check_sites(g, sites, "sites"));
  if (logits->rank != 2 || logits->shape[0] != B || logits->shape[1] != n_labels)
    return fail(TN_ERR_SHAPE_MISMATCH, "logits must be [B, n_labels]");
  if (prec != TN_PREC_FP32 && prec != TN_PREC_SPLIT_BF16) return fail(TN_ERR_UNSUPPORTED, "classifier precision %d", prec);
  WsLayout w = ws_layout(g);
  if (!workspace || ws_bytes < w.total) return fail(TN_ERR_WORKSPACE_TOO_SMALL, "workspace needs %zu bytes", w.total);
  hipStream_t st = static_cast<hipStream_t>(stream);
  char* ws = static_cast<char*>(workspace);
  float* ck = ckpt;
  // without a checkpoint buffer the two slots per chain live in the workspace
  float* local[2] = {reinterpret_cast<float*>(ws + w.vtmp0), reinterpret_cast<float*>(ws + w.vtmp1)};
  const float* px = static_cast<const float*>(pixels->data);
  const float* vc;
  const float* uc;
  if (ck) {
    TN_TRY(forward_core(g, sites, px, ck, st));
    vc = ck + (g.left_b.size() - 1) * g.vb;
    uc = ck + (g.left_b.size() + g.right_b.size() - 1) * g.vb;
  } else {
    // whole chains in runs of at most kMaxSeg sites, ping-ponging between two blocks
    const float* prev = nullptr;
    int k = 0, slot = 0;
    while (k < g.c) {
      const int n = std::min(kMaxSeg, g.c - k);
      TN_TRY(launch_chain(g, sites, px, 0, k, 1, n, prev, local[slot], nullptr, 1, st));
      prev = local[slot];
      slot ^= 1;
      k += n;
    }
    vc = prev;
    float* uloc[2] = {reinterpret_cast<float*>(ws + w.seg_v[0]), reinterpret_cast<float*>(ws + w.seg_g[0])};
    prev = nullptr;
    int t = g.N;
    slot = 0;
    while (t > g.c + 1) {
      const int n = std::min(kMaxSeg, t - (g.c + 1));
      TN_TRY(launch_chain(g, sites, px, 1, t - 1, -1, n, prev, uloc[slot], nullptr, 1, st));
      prev = uloc[slot];
      slot ^= 1;
      t -= n;
    }
    uc = prev;
  }
  // label site
  float* xbuf = reinterpret_cast<float*>(ws + w.xbuf);
  float* tbuf = reinterpret_cast<float*>(ws + w.tbuf);
  hipLaunchKernelGGL(expand_kernel, dim3(blocks_of((int64_t)B * chi * 2)), dim3(256), 0, st, vc, (const float*)nullptr,
                     px, n_sites, label_site, B, g.pad_chi, chi, xbuf);
  TN_TRY(hip_check(hipGetLastError(), "expand"));
  TN_TRY(label_t(g, sites[label_site], xbuf, tbuf, prec, st));
  hipLaunchKernelGGL(logits_kernel, dim3(blocks_of((int64_t)B * n_labels)), dim3(256), 0, st, tbuf, uc, vc, B, n_labels,
                     g.pad_chi, chi, static_cast<float*>(logits->data), logits->stride[0], logits->stride[1]);
  return hip_check(hipGetLastError(), "logits");
}

int32_t tn_mps_classifier_backward(int32_t n_sites, int32_t label_site, int32_t n_labels, const tn_tensor* sites,
                                   const tn_tensor* pixels, const float* ckpt, int32_t ckpt_every,
                                   const tn_tensor* dlogits, tn_tensor* dsites, void* workspace, size_t ws_bytes,
                                   int32_t prec, void* stream) {
  TN_TRY(check_tensor(pixels, "pixels", TN_F32));
  TN_TRY(check_tensor(dlogits, "dlogits", TN_F32));
  if (!ckpt) return fail(TN_ERR_INVALID_ARGUMENT, "the backward needs the forward's checkpoints");
  if (pixels->rank != 2 || pixels->shape[1] != n_sites || pixels->stride[1] != 1 || pixels->stride[0] != n_sites)
    return fail(TN_ERR_SHAPE_MISMATCH, "pixels must be a contiguous [B, n_sites] tensor");
  const int B = (int)pixels->shape[0];
  if (n_sites < 3 || !sites || !dsites) return fail(TN_ERR_INVALID_ARGUMENT, "need n_sites >= 3, sites and dsites");
  const int chi = (int)sites[1].shape[0];
  Geometry g;
  TN_TRY(geometry(n_sites, label_site, n_labels, B, chi, ckpt_every, g));
  TN_TRY(check_sites(g, sites, "sites"));
  for (int k = 0; k < n_sites; ++k) {
    char nm[32];
    snprintf(nm, sizeof(nm), "dsites[%d]", k);
    TN_TRY(check_tensor(&dsites[k], nm, TN_F32));
    if (dsites[k].rank != sites[k].rank) return fail(TN_ERR_SHAPE_MISMATCH, "%s has the wrong rank", nm);
    for (int q = 0; q < sites[k].rank; ++q)
      if (dsites[k].shape[q] != sites[k].shape[q]) return fail(TN_ERR_SHAPE_MISMATCH, "%s has the wrong shape", nm);
  }
  if (dlogits->rank != 2 || dlogits->shape[0] != B || dlogits->shape[1] != n_labels)
    return fail(TN_ERR_SHAPE_MISMATCH, "dlogits must be [B, n_labels]");
  if (prec != TN_PREC_FP32 && prec != TN_PREC_SPLIT_BF16) return fail(TN_ERR_UNSUPPORTED, "classifier precision %d", prec);
  WsLayout w = ws_layout(g);
  if (!workspace || ws_bytes < w.total) return fail(TN_ERR_WORKSPACE_TOO_SMALL, "workspace needs %zu bytes", w.total);
  hipStream_t st = static_cast<hipStream_t>(stream);
  char* ws = static_cast<char*>(workspace);
  const float* px = static_cast<const float*>(pixels->data);
  const float* gl = static_cast<const float*>(dlogits->data);
  const int64_t gs0 = dlogits->stride[0], gs1 = dlogits->stride[1];
  const int64_t vb = g.vb;
  const int pc = g.pad_chi;
  const float* vc = ckpt + (g.left_b.size() - 1) * vb;
  const float* uc = ckpt + (g.left_b.size() + g.right_b.size() - 1) * vb;
  float* xbuf = reinterpret_cast<float*>(ws + w.xbuf);
  float* tbuf = reinterpret_cast<float*>(ws + w.tbuf);
  float* ybuf = reinterpret_cast<float*>(ws + w.ybuf);
  float* gubuf = reinterpret_cast<float*>(ws + w.gubuf);
  float* abar = reinterpret_cast<float*>(ws + w.vtmp0);   // adjoint of the left vector
  float* ubar = reinterpret_cast<float*>(ws + w.vtmp1);   // adjoint of the right vector
  float* segv[2] = {reinterpret_cast<float*>(ws + w.seg_v[0]), reinterpret_cast<float*>(ws + w.seg_v[1])};
  float* segg[2] = {reinterpret_cast<float*>(ws + w.seg_g[0]), reinterpret_cast<float*>(ws + w.seg_g[1])};
  float* xseg[2] = {reinterpret_cast<float*>(ws + w.xseg[0]), reinterpret_cast<float*>(ws + w.xseg[1])};
  float* gbuf[2] = {reinterpret_cast<float*>(ws + w.gbuf[0]), reinterpret_cast<float*>(ws + w.gbuf[1])};
  const tn_tensor& ac = sites[label_site];

  // ---- label site
  hipLaunchKernelGGL(expand_kernel, dim3(blocks_of((int64_t)B * chi * 2)), dim3(256), 0, st, vc, (const float*)nullptr,
                     px, n_sites, label_site, B, pc, chi, xbuf);
  TN_TRY(label_t(g, ac, xbuf, tbuf, prec, st));
  // dA_c[a, s, l, z] = sum_b Xc[b, a, s] (g[b, l] u[b, z] 2^(e_v + e_u))
  hipLaunchKernelGGL(gu_kernel, dim3(blocks_of((int64_t)B * n_labels * chi)), dim3(256), 0, st, gl, gs0, gs1, uc, vc, B,
                     n_labels, pc, chi, gubuf);
  {
    tn_tensor xv = make_view(xbuf, TN_F32, {B, chi, 2});
    tn_tensor gv = make_view(gubuf, TN_F32, {B, n_labels, chi});
    const int32_t pa[1] = {0}, pb[1] = {0};
    TN_TRY(contract_between_impl(&xv, &gv, 1, pa, pb, &dsites[label_site], nullptr, 0, prec, st));
  }
  // abar_c[b, a] = sum_s Phi_s sum_{l z} A_c[a, s, l, z] g[b, l] u[b, z]   (exponent e_u)
  hipLaunchKernelGGL(gu_kernel, dim3(blocks_of((int64_t)B * n_labels * chi)), dim3(256), 0, st, gl, gs0, gs1, uc,
                     (const float*)nullptr, B, n_labels, pc, chi, gubuf);
  {
    tn_tensor gv = make_view(gubuf, TN_F32, {B, n_labels, chi});
    tn_tensor yv = make_view(ybuf, TN_F32, {B, chi, 2});
    const int32_t pa[2] = {1, 2}, pb[2] = {2, 3};
    TN_TRY(contract_between_impl(&gv, &ac, 2, pa, pb, &yv, nullptr, 0, prec, st));
  }
  hipLaunchKernelGGL(phi_contract_kernel, dim3(blocks_of((int64_t)B * pc)), dim3(256), 0, st, ybuf, px, n_sites,
                     label_site, B, chi, pc, uc, abar);
  // ubar_{c+1}[b, z] = sum_l g[b, l] T[b, l, z]   (exponent e_v)
  hipLaunchKernelGGL(gt_kernel, dim3(blocks_of((int64_t)B * pc)), dim3(256), 0, st, gl, gs0, gs1, tbuf, B, n_labels,
                     chi, pc, vc, ubar);
  TN_TRY(hip_check(hipGetLastError(), "label site"));

  // ---- chains, segment by segment from the label site outwards; round r
  // takes left segment nl-1-r and right segment nr-1-r.  Per side: one
  // launch recomputes the segment's vectors from its checkpoint and carries
  // the adjoint through it (the two are independent), then the segment's
  // weight gradients.
  const int nl = (int)g.left_b.size() - 1, nr = (int)g.right_b.size() - 1;
  const size_t off = g.left_b.size();
  for (int r = 0; r < std::max(nl, nr); ++r) {
    std::vector<ChainArgs> runs;
    int jl = nl - 1 - r, jr = nr - 1 - r;
    if (jl >= 0) {
      const int s0 = g.left_b[jl], s1 = g.left_b[jl + 1], n = s1 - s0;
      const float* ck = jl == 0 ? nullptr : ckpt + jl * vb;
      // v_{s0} .. v_{s1-1}: step i stores the input of site s0 + i
      runs.push_back(chain_args(g, sites, px, 0, s0, 1, n, ck, nullptr, segv[0], 1));
      // abar_{s1} -> abar_{s0}: step i at site s1-1-i stores abar_{s1-i}
      runs.push_back(chain_args(g, sites, px, 1, s1 - 1, -1, n, abar, abar, segg[0], 0));
    }
    if (jr >= 0) {
      const int t0 = g.right_b[jr], t1 = g.right_b[jr + 1], n = t0 - t1;   // sites t1 .. t0-1
      const float* ck = jr == 0 ? nullptr : ckpt + (off + jr) * vb;
      // u_{t0} .. u_{t1+1}: step i at site t0-1-i stores u_{t0-i}
      runs.push_back(chain_args(g, sites, px, 1, t0 - 1, -1, n, ck, nullptr, segv[1], 1));
      // ubar_{t1} -> ubar_{t0}: step i at site t1+i stores ubar_{t1+i}
      runs.push_back(chain_args(g, sites, px, 0, t1, 1, n, ubar, ubar, segg[1], 0));
    }
    TN_TRY(launch_chains(g, runs, st));
    if (jl >= 0) {
      // site k = s1-1-j:  X from v_k (segv slot n-1-j), G = abar_{k+1} (segg slot j)
      const int s0 = g.left_b[jl], s1 = g.left_b[jl + 1];
      TN_TRY(segment_grads(g, segv[0], segg[0], s1 - s0, s1 - 1, px, xseg[0], gbuf[0], dsites, prec, st));
    }
    if (jr >= 0) {
      // site k = t0-1-j:  X from ubar_k (segg slot n-1-j), G = u_{k+1} (segv slot j)
      const int t0 = g.right_b[jr], t1 = g.right_b[jr + 1];
      TN_TRY(segment_grads(g, segg[1], segv[1], t0 - t1, t0 - 1, px, xseg[1], gbuf[1], dsites, prec, st));
    }
  }
  return TN_OK;
}

int32_t tn_softmax_xent(const tn_tensor* logits, const int64_t* labels, int32_t batch, double* loss, tn_tensor* dlogits,
                        void* workspace, size_t ws_bytes, void* stream) {
  TN_TRY(check_tensor(logits, "logits", TN_F32));
  TN_TRY(check_tensor(dlogits, "dlogits", TN_F32));
  if (!labels || !loss) return fail(TN_ERR_INVALID_ARGUMENT, "labels and loss must be given");
  if (logits->rank != 2 || logits->shape[0] != batch || dlogits->rank != 2 || dlogits->shape[0] != batch ||
      dlogits->shape[1] != logits->shape[1])
    return fail(TN_ERR_SHAPE_MISMATCH, "logits and dlogits must be [batch, n_labels]");
  if (!workspace || ws_bytes < (size_t)batch * 8) return fail(TN_ERR_WORKSPACE_TOO_SMALL, "workspace needs %d bytes", batch * 8);
  hipStream_t st = static_cast<hipStream_t>(stream);
  double* part = static_cast<double*>(workspace);
  hipLaunchKernelGGL(softmax_xent_kernel, dim3((batch + 255) / 256), dim3(256), 0, st,
                     static_cast<const float*>(logits->data), logits->stride[0], logits->stride[1], labels, batch,
                     (int)logits->shape[1], part, static_cast<float*>(dlogits->data), dlogits->stride[0],
                     dlogits->stride[1]);
  hipLaunchKernelGGL(mean_kernel, dim3(1), dim3(256), 0, st, part, batch, loss);
  return hip_check(hipGetLastError(), "softmax xent");
}

}  // extern "C"
