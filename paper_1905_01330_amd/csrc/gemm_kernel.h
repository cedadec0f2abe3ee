// Tiled matrix-core contraction kernel for gfx950 (CDNA4).
//
// C[m, n] = sum_k A[m, k] B[k, n] where A, B and C are arbitrary strided
// views (the M, N and K indices are groups of tensor axes).  The index
// permutation of a tensordot happens inside the global -> LDS gather: each
// thread reads a 1x4 (k-contiguous) or 4x4 (m/n-contiguous, transposed in
// registers) micro-block and writes it to LDS in the layout the MFMA operand
// reads want (8 consecutive k per lane).  No separate transpose pass exists.
//
// Precisions: FP32 operands on v_mfma_f32_32x32x2_f32; BF16 operands on
// v_mfma_f32_32x32x16_bf16; the compensated split keeps 2 or 3 BF16 terms
// per operand in separate LDS planes and issues 3 or 6 term products per
// k-step into the same FP32 accumulator registers.
#pragma once

#include "common.h"

namespace tn {

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4_t __attribute__((ext_vector_type(4)));
typedef float f32x16_t __attribute__((ext_vector_type(16)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));
// the same with only 4-byte alignment: gfx950 runs 16-byte global loads at
// any 4-byte-aligned address, so a row of an odd-sized operand that starts
// anywhere is still read with one load per four elements
typedef float f32x4u_t __attribute__((ext_vector_type(4), aligned(4)));

__device__ __forceinline__ f32x4_t load4u(const float* p) { return *reinterpret_cast<const f32x4u_t*>(p); }

enum Prec : int { P_FP32 = 0, P_BF16 = 1, P_X6 = 2, P_X3 = 3 };

template <int P>
struct PrecInfo {
  static constexpr int planes = (P == P_X6) ? 3 : (P == P_X3 ? 2 : 1);
  static constexpr bool bf = (P != P_FP32);
  // term products (i, j), smallest first, all into one accumulator
  static constexpr int nprod = (P == P_X6) ? 6 : (P == P_X3 ? 3 : 1);
};

__device__ constexpr int prod_a(int P, int q) {
  // x6: (1,1) (0,2) (2,0) (0,1) (1,0) (0,0);  x3: (0,1) (1,0) (0,0)
  return P == P_X6 ? (q == 0 ? 1 : q == 1 ? 0 : q == 2 ? 2 : q == 3 ? 0 : q == 4 ? 1 : 0)
       : P == P_X3 ? (q == 0 ? 0 : q == 1 ? 1 : 0)
                   : 0;
}
__device__ constexpr int prod_b(int P, int q) {
  return P == P_X6 ? (q == 0 ? 1 : q == 1 ? 2 : q == 2 ? 0 : q == 3 ? 1 : q == 4 ? 0 : 0)
       : P == P_X3 ? (q == 0 ? 1 : q == 1 ? 0 : 0)
                   : 0;
}

// exact power-of-two rescale factor 2^-e for a max-abs bit pattern (1 if unusable)
__device__ inline float pow2_inverse_scale(uint32_t bits) {
  uint32_t e = (bits >> 23) & 0xffu;
  if (e == 0u || e > 253u) return 1.0f;
  return __uint_as_float((254u - e) << 23);
}

template <int P, int R, int BK>
struct LdsOperand {
  static constexpr int LDK = BK + 4;   // fp32 row pitch (floats)
  static constexpr int LDH = BK;       // bf16 row pitch (elements): unpadded, see bf16_slot
  static constexpr int bytes = PrecInfo<P>::bf ? R * LDH * 2 * PrecInfo<P>::planes : R * LDK * 4;
};

// Element offset of (row, k) in an unpadded BF16 plane with BK elements per
// row.  The plane is cut into 16-row groups; row r = 16q + 4a + m of a group
// is placed in a permuted row slot and its 16-byte chunks (8 k each) are
// XOR-swizzled, so that every access pattern of the kernel is free of bank
// conflicts.  The rules were measured on gfx950 with the bank-conflict
// counter: 4-byte stores are served 32 lanes per cycle over 32 banks of 4
// bytes, 8-byte stores 16 lanes over 32 banks, 16-byte loads 16 lanes over
// 64 banks (two-address stores run as two independent passes).  Patterns:
//   - MFMA fragment loads: 16 consecutive rows, one chunk each (16 bytes);
//   - k-contiguous gathers: 4 consecutive rows, 4 k per lane (8 bytes);
//   - transposed gathers: rows 4g + i for 4 consecutive g, 2 k (4 bytes) or
//     4 k (8 bytes) per lane.
// Stores need distinct 32-bank windows (slot mod 4, 2, 1 for BK = 16, 32,
// 64): a Latin square in (a, m).  Loads need distinct 64-bank quads across
// 16 rows, which the high slot bits and the chunk swizzle provide.
template <int BK>
__device__ __forceinline__ int bf16_slot(int row, int k) {
  const int q = row >> 4, a = (row >> 2) & 3, m = row & 3;
  int slot, sw;
  if constexpr (BK == 16) {         // 2 chunks per row
    slot = 16 * q + 8 * (a & 1) + 4 * (a >> 1) + ((a + m) & 3);
    sw = a & 1;
  } else if constexpr (BK == 32) {  // 4 chunks per row
    slot = 16 * q + 4 * m + ((a + m) & 3);
    sw = m;
  } else {                          // BK == 64: 8 chunks per row
    static_assert(BK == 64, "BF16 LDS layout is defined for BK = 16, 32, 64");
    slot = row;
    sw = (row >> 1) & 7;
  }
  return slot * BK + ((((k >> 3) ^ sw)) << 3) + (k & 7);
}

typedef float f32x2_t __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
typedef uint32_t u32x2_t __attribute__((ext_vector_type(2)));

// Split two FP32 values into BF16 terms x = x0 + x1 + x2 (each rounded to
// nearest even; exact for normal inputs).  The pair is converted with one
// packed conversion per term; the terms come back packed two to a dword.
template <int NPL>
__device__ __forceinline__ void split_pair(float a, float b, uint32_t (&t)[3]) {
  f32x2_t x = {a, b};
  uint32_t u = __builtin_bit_cast(uint32_t, __builtin_convertvector(x, bf16x2_t));
  t[0] = u;
  if constexpr (NPL >= 2) {
    const float ra = a - __uint_as_float(u << 16);
    const float rb = b - __uint_as_float(u & 0xffff0000u);
    f32x2_t r = {ra, rb};
    u = __builtin_bit_cast(uint32_t, __builtin_convertvector(r, bf16x2_t));
    t[1] = u;
    if constexpr (NPL >= 3) {
      f32x2_t r2 = {ra - __uint_as_float(u << 16), rb - __uint_as_float(u & 0xffff0000u)};
      t[2] = __builtin_bit_cast(uint32_t, __builtin_convertvector(r2, bf16x2_t));
    }
  }
}

template <int P, int R, int BK>
__device__ inline void lds_put4(char* base, int row, int kcol, f32x4_t v) {
  if constexpr (!PrecInfo<P>::bf) {
    float* p = reinterpret_cast<float*>(base);
    *reinterpret_cast<f32x4_t*>(p + row * LdsOperand<P, R, BK>::LDK + kcol) = v;
  } else {
    constexpr int NPL = PrecInfo<P>::planes;
    constexpr int plane = R * LdsOperand<P, R, BK>::LDH;
    __bf16* h = reinterpret_cast<__bf16*>(base) + bf16_slot<BK>(row, kcol);
    uint32_t lo[3], hi[3];
    split_pair<NPL>(v[0], v[1], lo);
    split_pair<NPL>(v[2], v[3], hi);
#pragma unroll
    for (int p = 0; p < NPL; ++p) {
      u32x2_t w = {lo[p], hi[p]};
      *reinterpret_cast<u32x2_t*>(h + p * plane) = w;
    }
  }
}

// Two consecutive k of one row (the 4 x 2 transposed micro-block)
template <int P, int R, int BK>
__device__ inline void lds_put2(char* base, int row, int kcol, float v0, float v1) {
  if constexpr (!PrecInfo<P>::bf) {
    float* p = reinterpret_cast<float*>(base);
    f32x2_t w = {v0, v1};
    *reinterpret_cast<f32x2_t*>(p + row * LdsOperand<P, R, BK>::LDK + kcol) = w;
  } else {
    constexpr int NPL = PrecInfo<P>::planes;
    constexpr int plane = R * LdsOperand<P, R, BK>::LDH;
    __bf16* h = reinterpret_cast<__bf16*>(base) + bf16_slot<BK>(row, kcol);
    uint32_t t[3];
    split_pair<NPL>(v0, v1, t);
#pragma unroll
    for (int p = 0; p < NPL; ++p) *reinterpret_cast<uint32_t*>(h + p * plane) = t[p];
  }
}

// Per-thread gather of one operand tile (R rows x BK k) per stage.
//   which = 0: operand A (rows = M, strides gm.s[0], gk.s[0])
//   which = 1: operand B (rows = N, strides gn.s[0], gk.s[1])
template <int P, int R, int BK, int NT, int KIDX>
struct OperandLoader {
  static constexpr int KQ = BK / 4;
  static constexpr int NKV = R * BK / 4;
  static constexpr int NMV = R * BK / 16;
  static constexpr int VK = (NKV + NT - 1) / NT;
  static constexpr int VM = (NMV + NT - 1) / NT;
  static constexpr int NREG = (VK > 4 * VM) ? VK : 4 * VM;
  static constexpr int NROW = (VK > VM) ? VK : VM;

  f32x4_t st[NREG];
  int64_t rowoff[NROW];
  uint32_t rowok;
  int mode;
  const float* base;
  int K;
  int nrows;
  int row0;
  float scale;

  // offset of contracted index k: one multiply for a single merged axis, else
  // a short (not unrolled) digit loop, so the callers' loops stay unrollable
  __device__ static inline int64_t koff(const Group& gk, int k) {
    if (gk.n == 1) return (int64_t)k * gk.s[KIDX][0];
    int64_t o = 0;
    uint32_t idx = (uint32_t)k;
#pragma unroll 1
    for (int i = gk.n - 1; i >= 0; --i) {
      uint32_t q = fast_div(idx, gk.mul[i], gk.shr[i]);
      o += (int64_t)(idx - q * gk.dim[i]) * gk.s[KIDX][i];
      idx = q;
    }
    return o;
  }

  __device__ __forceinline__ void init(int mode_, const float* base_, const Group& grows, int row0_, int nrows_, int K_,
                              float scale_) {
    mode = mode_;
    base = base_;
    K = K_;
    nrows = nrows_;
    row0 = row0_;
    scale = scale_;
    rowok = 0;
    const int tid = threadIdx.x;
    if (mode != LOAD_MNVEC) {
#pragma unroll
      for (int v = 0; v < VK; ++v) {
        int idx = tid + v * NT;
        int row = row0 + (mode == LOAD_MNSCALAR ? idx % R : idx / KQ);
        rowoff[v] = 0;
        if (idx < NKV && row < nrows) {
          int64_t o[1];
          group_offsets<1>(grows, (uint32_t)row, o, 0);
          rowoff[v] = o[0];
          rowok |= 1u << v;
        }
      }
    } else {
#pragma unroll
      for (int v = 0; v < VM; ++v) {
        int idx = tid + v * NT;
        int row = row0 + (idx / KQ) * 4;
        rowoff[v] = 0;
        if (idx < NMV && row < nrows) {
          int64_t o[1];
          group_offsets<1>(grows, (uint32_t)row, o, 0);
          rowoff[v] = o[0];
          rowok |= 1u << v;
        }
      }
    }
  }

  __device__ __forceinline__ void load(int k0, const Group& gk) {
    const int tid = threadIdx.x;
    if (mode == LOAD_KVEC) {
#pragma unroll
      for (int v = 0; v < VK; ++v) {
        int idx = tid + v * NT;
        int k = k0 + (idx % KQ) * 4;
        f32x4_t x = {0.f, 0.f, 0.f, 0.f};
        if (((rowok >> v) & 1u) && k < K) {
          // a partial last micro-block (K % 4 != 0, one contracted axis)
          // is read element by element
          const float* p = base + rowoff[v] + koff(gk, k);
          if (k + 4 <= K) {
            x = load4u(p);
          } else {
#pragma unroll
            for (int j = 0; j < 3; ++j)
              if (k + j < K) x[j] = p[j];
          }
        }
        st[v] = x;
      }
    } else if ((mode == LOAD_MNSCALAR || mode == LOAD_GENERIC) && gk.n == 1) {
      // one contracted axis: one offset per micro-block, its four k at
      // multiples of the stride (the scalar gathers of both forms below)
      const int64_t sk = gk.s[KIDX][0];
      const bool full = k0 + BK <= K;   // every k of the stage in range: no per-element checks
#pragma unroll
      for (int v = 0; v < VK; ++v) {
        int idx = tid + v * NT;
        int k = k0 + (mode == LOAD_MNSCALAR ? idx / R : idx % KQ) * 4;
        f32x4_t x = {0.f, 0.f, 0.f, 0.f};
        if ((rowok >> v) & 1u) {
          const float* p = base + rowoff[v] + (int64_t)k * sk;
          if (full) {
#pragma unroll
            for (int j = 0; j < 4; ++j) x[j] = p[j * sk];
          } else {
#pragma unroll
            for (int j = 0; j < 4; ++j)
              if (k + j < K) x[j] = p[j * sk];
          }
        }
        st[v] = x;
      }
    } else if (mode == LOAD_MNSCALAR) {
      // lanes run along the unit-stride rows: each load instruction reads
      // 64 consecutive floats of one k
#pragma unroll
      for (int v = 0; v < VK; ++v) {
        int idx = tid + v * NT;
        int k = k0 + (idx / R) * 4;
        f32x4_t x = {0.f, 0.f, 0.f, 0.f};
        if ((rowok >> v) & 1u) {
#pragma unroll
          for (int j = 0; j < 4; ++j)
            if (k + j < K) x[j] = base[rowoff[v] + koff(gk, k + j)];
        }
        st[v] = x;
      }
    } else if (mode == LOAD_GENERIC) {
#pragma unroll
      for (int v = 0; v < VK; ++v) {
        int idx = tid + v * NT;
        int k = k0 + (idx % KQ) * 4;
        f32x4_t x = {0.f, 0.f, 0.f, 0.f};
        if ((rowok >> v) & 1u) {
#pragma unroll
          for (int j = 0; j < 4; ++j)
            if (k + j < K) x[j] = base[rowoff[v] + koff(gk, k + j)];
        }
        st[v] = x;
      }
    } else {
#pragma unroll
      for (int v = 0; v < VM; ++v) {
        int idx = tid + v * NT;
        int k = k0 + (idx % KQ) * 4;
        // the four k of the micro-block: one offset and the innermost stride
        // when they share the innermost K run, else one offset each
        const int last = gk.n - 1;
        const int64_t ko = k < K ? koff(gk, k) : 0;
        const bool run = gk.n == 1 || (k % (int)gk.dim[last]) + 3 < (int)gk.dim[last];
        const int64_t ks = gk.s[KIDX][last];
        const bool ok = (rowok >> v) & 1u;
        f32x4_t x0 = {0.f, 0.f, 0.f, 0.f}, x1 = x0, x2 = x0, x3 = x0;
        // a partial last block of rows (one row axis, M % 4 != 0): element by
        // element, rows past the end read as zero
        const int nv = nrows - (row0 + (idx / KQ) * 4);
        if (ok && nv < 4) {
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            if (k + j >= K) continue;
            const float* p = base + rowoff[v] + koff(gk, k + j);
            f32x4_t y = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int i = 0; i < 3; ++i)
              if (i < nv) y[i] = p[i];
            if (j == 0) x0 = y;
            else if (j == 1) x1 = y;
            else if (j == 2) x2 = y;
            else x3 = y;
          }
        } else if (run) {
          const float* p = base + rowoff[v] + ko;
          if (ok && k + 0 < K) x0 = load4u(p);
          if (ok && k + 1 < K) x1 = load4u(p + ks);
          if (ok && k + 2 < K) x2 = load4u(p + 2 * ks);
          if (ok && k + 3 < K) x3 = load4u(p + 3 * ks);
        } else {
          if (ok && k + 0 < K) x0 = load4u(base + rowoff[v] + koff(gk, k + 0));
          if (ok && k + 1 < K) x1 = load4u(base + rowoff[v] + koff(gk, k + 1));
          if (ok && k + 2 < K) x2 = load4u(base + rowoff[v] + koff(gk, k + 2));
          if (ok && k + 3 < K) x3 = load4u(base + rowoff[v] + koff(gk, k + 3));
        }
        st[4 * v + 0] = x0;
        st[4 * v + 1] = x1;
        st[4 * v + 2] = x2;
        st[4 * v + 3] = x3;
      }
    }
  }

  __device__ __forceinline__ void store(char* lds) {
    const int tid = threadIdx.x;
    if (mode == LOAD_MNSCALAR) {
#pragma unroll
      for (int v = 0; v < VK; ++v) {
        int idx = tid + v * NT;
        if (idx < NKV) lds_put4<P, R, BK>(lds, idx % R, (idx / R) * 4, st[v]);
      }
    } else if (mode != LOAD_MNVEC) {
#pragma unroll
      for (int v = 0; v < VK; ++v) {
        int idx = tid + v * NT;
        if (idx < NKV) lds_put4<P, R, BK>(lds, idx / KQ, (idx % KQ) * 4, st[v]);
      }
    } else {
#pragma unroll
      for (int v = 0; v < VM; ++v) {
        int idx = tid + v * NT;
        if (idx < NMV) {
          int r0 = (idx / KQ) * 4;
          int kc = (idx % KQ) * 4;
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            f32x4_t t = {st[4 * v + 0][i], st[4 * v + 1][i], st[4 * v + 2][i], st[4 * v + 3][i]};
            lds_put4<P, R, BK>(lds, r0 + i, kc, t);
          }
        }
      }
    }
  }
};

// Fast gather for a single merged contracted axis (the common case after
// axis merging): each thread keeps one pointer per micro-block that advances
// by a constant every stage; rows past the end are clamped to the last valid
// row (their products only reach output rows that are never stored), so
// only the last, partial K stage carries bounds checks.
//   MODE = LOAD_KVEC : k is the unit-stride axis, 1 x 4 micro-blocks
//   MODE = LOAD_MNVEC: the row axis is unit-stride, 4 x 4 micro-blocks,
//                      transposed in registers before the LDS store
template <int P, int R, int BK, int NT, int MODE, int DEPTH = 2>
struct FastLoader {
  // m/n-contiguous operands are read as 4 rows x KD k micro-blocks (KD float4
  // loads, transposed in registers).  KD = 4 when the 4 x 4 blocks cover the
  // workgroup evenly, else KD = 2 so that no thread idles.
  static constexpr int KD = (MODE == LOAD_KVEC || (R * BK / 16) % NT == 0 || (R * BK / 8) % NT != 0) ? 4 : 2;
  static constexpr int KQ = MODE == LOAD_KVEC ? BK / 4 : BK / KD;
  static constexpr int NMB = MODE == LOAD_KVEC ? R * BK / 4 : R * BK / (4 * KD);
  static constexpr int NV = (NMB + NT - 1) / NT;
  static constexpr bool EXACT = NMB % NT == 0;
  static constexpr int NREG = MODE == LOAD_KVEC ? NV : KD * NV;

  f32x4_t st[DEPTH][NREG];   // DEPTH stages in flight (set = stage parity)
  const float* ptr[NV];
  int kq[NV];
  int64_t sk;
  int K;
  int row0, nrows;

  __device__ __forceinline__ void init(const float* base, const Group& grows, int row0_, int nrows_, int64_t sk_, int K_) {
    sk = sk_;
    K = K_;
    row0 = row0_;
    nrows = nrows_;
    const int tid = threadIdx.x;
    (void)tid;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      const int idx = block_of(v);
      int row, k;
      if constexpr (MODE == LOAD_KVEC) {
        row = row0 + idx / KQ;
        k = (idx % KQ) * 4;
        row = row < nrows ? row : nrows - 1;
      } else {
        // k-chunk fastest: a wavefront's transposed LDS writes land in
        // distinct banks while its global reads stay 128-byte runs per k row
        row = row0 + (idx / KQ) * 4;
        k = (idx % KQ) * KD;
        // a block past the end re-reads the last whole one (its LDS rows
        // are past M and never stored); M >= 4
        row = row < nrows ? row : nrows - 4;
      }
      int64_t o[1];
      group_offsets<1>(grows, (uint32_t)row, o, 0);
      kq[v] = k;
      ptr[v] = base + o[0] + (int64_t)k * sk;
    }
  }

  // slot v of a thread covers micro-block idx; past the last block it repeats
  // block idx % NMB (the same load and the same LDS store of the same value
  // as another slot), which keeps the stage free of branches
  __device__ static __forceinline__ int block_of(int v) {
    const int idx = threadIdx.x + v * NT;
    return (EXACT || idx < NMB) ? idx : idx % NMB;
  }

  // slot v of the stage starting at k0 into register set SET
  template <bool TAIL, int SET>
  __device__ __forceinline__ void load_slot(int k0, int v) {
    if constexpr (MODE == LOAD_KVEC) {
      f32x4_t x = {0.f, 0.f, 0.f, 0.f};
      if constexpr (!TAIL) {
        x = load4u(ptr[v]);
      } else {
        // the stage's micro-blocks past K are zero; a partial one (K % 4
        // != 0) is read element by element
        const int k = k0 + kq[v];
        if (k + 4 <= K) {
          x = load4u(ptr[v]);
        } else {
#pragma unroll
          for (int j = 0; j < 3; ++j)
            if (k + j < K) x[j] = ptr[v][j];
        }
      }
      st[SET][v] = x;
    } else {
#pragma unroll
      for (int j = 0; j < KD; ++j) {
        f32x4_t x = {0.f, 0.f, 0.f, 0.f};
        if constexpr (!TAIL) {
          // a partial last block of rows (M % 4 != 0) reads up to three
          // elements past row M - 1 of this k: inside the view, since no
          // stage but the last holds k = K - 1 and the k stride is >= 4
          x = load4u(ptr[v] + j * sk);
        } else if (k0 + kq[v] + j < K) {
          // the last stage reads a partial block element by element
          const int nv = nrows - (row0 + (block_of(v) / KQ) * 4);
          if (nv >= 4 || nv <= 0) {
            x = load4u(ptr[v] + j * sk);
          } else {
#pragma unroll
            for (int i = 0; i < 3; ++i)
              if (i < nv) x[i] = ptr[v][j * sk + i];
          }
        }
        st[SET][KD * v + j] = x;
      }
    }
    ptr[v] += BK * sk;
  }

  template <bool TAIL, int SET>
  __device__ __forceinline__ void load(int k0) {
#pragma unroll
    for (int v = 0; v < NV; ++v) load_slot<TAIL, SET>(k0, v);
  }

  // stage kt (k0 = kt * BK) into register set SET, if the stage exists;
  // the last stage (partial or not) takes the careful loads
  template <int SET>
  __device__ __forceinline__ void load_stage(int kt, int nk) {
    if (kt < nk - 1)
      load<false, SET>(kt * BK);
    else if (kt == nk - 1)
      load<true, SET>(kt * BK);
  }

  // split slot v of register set SET and store it into the LDS stage `lds`
  template <int SET>
  __device__ __forceinline__ void store_slot(char* lds, int v) {
    const int idx = block_of(v);
    if constexpr (MODE == LOAD_KVEC) {
      lds_put4<P, R, BK>(lds, idx / KQ, (idx % KQ) * 4, st[SET][v]);
    } else {
      const int r0 = (idx / KQ) * 4;
      const int kc = (idx % KQ) * KD;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        if constexpr (KD == 4) {
          f32x4_t t = {st[SET][4 * v + 0][i], st[SET][4 * v + 1][i], st[SET][4 * v + 2][i], st[SET][4 * v + 3][i]};
          lds_put4<P, R, BK>(lds, r0 + i, kc, t);
        } else {
          lds_put2<P, R, BK>(lds, r0 + i, kc, st[SET][2 * v + 0][i], st[SET][2 * v + 1][i]);
        }
      }
    }
  }

  template <int SET>
  __device__ __forceinline__ void store(char* lds) {
#pragma unroll
    for (int v = 0; v < NV; ++v) store_slot<SET>(lds, v);
  }
};

// Copy an index group with static field accesses only (so a by-value kernel
// argument is never indexed dynamically, which would force a private copy).
__device__ __forceinline__ void copy_group(Group& dst, const Group& src) {
  if (threadIdx.x == 0) {
    dst.n = src.n;
#pragma unroll
    for (int i = 0; i < kMaxAxes; ++i) {
      dst.dim[i] = src.dim[i];
      dst.mul[i] = src.mul[i];
      dst.shr[i] = src.shr[i];
      dst.s[0][i] = src.s[0][i];
      dst.s[1][i] = src.s[1][i];
      dst.s[2][i] = src.s[2][i];
    }
  }
}

// XCD-aware tile order: the hardware deals workgroups round-robin over the 8
// XCDs, so consecutive ids are remapped to one XCD's contiguous range, then
// grouped by GROUP_M tile rows so neighbouring tiles share A rows and B
// columns in that XCD's L2.
__device__ inline void tile_coords(int bid, int tiles_m, int tiles_n, int& tm, int& tn) {
  const int T = tiles_m * tiles_n;
  int local = bid;
  if (T >= 16) {
    const int x = bid & 7, i = bid >> 3;
    const int q = T >> 3, r = T & 7;
    local = x * q + (x < r ? x : r) + i;
  }
  constexpr int GROUP_M = 8;
  const int per_group = GROUP_M * tiles_n;
  const int g = local / per_group;
  const int first_m = g * GROUP_M;
  const int gsize = (tiles_m - first_m) < GROUP_M ? (tiles_m - first_m) : GROUP_M;
  const int in_g = local - g * per_group;
  tm = first_m + in_g % gsize;
  tn = in_g / gsize;
}

// AMODE / BMODE: LOAD_KVEC or LOAD_MNVEC select the fast gathers (single
// merged K axis); -1 selects the run-time-mode gathers that handle any layout.
// WK > 1 slices every stage's k-chunks over WK groups of WM x WN waves (each
// group accumulates its share of K for the whole tile); the groups' sums are
// added through LDS before the store.
template <int P, int BM, int BN, int BK, int WM, int WN, int AMODE = -1, int BMODE = -1, int WK = 1>
struct GemmTile {
  static constexpr int NT = WM * WN * WK * 64;
  static constexpr int TM = BM / WM / 32;
  static constexpr int TN = BN / WN / 32;
  static constexpr int bytesA = LdsOperand<P, BM, BK>::bytes;
  static constexpr int bytesB = LdsOperand<P, BN, BK>::bytes;
  static constexpr int stage = bytesA + bytesB;
  // the k-slice groups' sums pass through LDS once the stages are done
  static constexpr int red_bytes = WK > 1 ? WM * WN * (BM / WM / 32) * (BN / WN / 32) * 16 * 64 * 4 : 0;
  static constexpr int lds_bytes = 2 * stage > red_bytes ? 2 * stage : red_bytes;
  static_assert(TM >= 1 && TN >= 1, "tile too small for 32x32 blocks");
  static_assert(BK % 16 == 0, "BK must be a multiple of 16");
  static_assert((BK / 16) % WK == 0, "every k-slice group needs whole 16-wide chunks");

  // stages summed into the temporary before it is added to the accumulator (64 k)
  static constexpr int FLUSH = BK >= 64 ? 1 : 64 / BK;
  // Wave tiles above four 32x32 blocks do not keep a temporary per block:
  // each block's term products of a stage form one zero-based chain that is
  // added to the accumulator at once (more VALU adds, half the registers).
  static constexpr bool CHAIN = PrecInfo<P>::planes > 1 && TM * TN > 4 && TM * TN * 16 + 32 <= 128;
  // global loads run DEPTH stages ahead; workgroups of eight waves (two per
  // SIMD by construction, a fixed 256-register budget) keep one stage ahead
  static constexpr int DEPTH = NT >= 512 ? 1 : 2;
  // parts `between` is cut into (one per 32-wide block of the wide side)
  static constexpr int NPARTS = CHAIN ? (TM >= TN ? TM : TN) : 1;
  static constexpr int TMT = PrecInfo<P>::planes > 1 && !CHAIN ? TM : 1;
  static constexpr int TNT = PrecInfo<P>::planes > 1 && !CHAIN ? TN : 1;

  __device__ static __forceinline__ void flush_tmp(f32x16_t (&acc)[TM][TN], f32x16_t (&tmp)[TMT][TNT]) {
    if constexpr (PrecInfo<P>::planes > 1 && !CHAIN) {
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) acc[i][j] += tmp[i][j];
    }
  }

  // One stage: read the operand fragments from LDS and run the MFMAs; the
  // callable `between(part)` (work independent of this stage: the next
  // stage's split and LDS stores, cut into NPARTS parts) runs interleaved
  // with the matrix-core ops.  Wide wave tiles call part b after the
  // products of their b-th 32-wide block are issued; the others call part 0
  // once the first fragments are read.
  struct Nothing {
    __device__ __forceinline__ void operator()(int) const {}
  };
  template <typename F = Nothing>
  __device__ static __forceinline__ void compute(const char* sa, const char* sb, f32x16_t (&acc)[TM][TN],
                                                 f32x16_t (&tmp)[TMT][TNT], bool first, bool flush, int wm_off,
                                                 int wn_off, int kslice, const F& between = F()) {
    compute_body(sa, sb, acc, tmp, first, flush, wm_off, wn_off, kslice, between);
  }

  template <typename F>
  __device__ static __forceinline__ void compute_body(const char* sa, const char* sb, f32x16_t (&acc)[TM][TN],
                                                      f32x16_t (&tmp)[TMT][TNT], bool first, bool flush, int wm_off,
                                                      int wn_off, int kslice, const F& between) {
    const int lane = threadIdx.x & 63;
    const int lr = lane & 31, lh = lane >> 5;
    if constexpr (!PrecInfo<P>::bf) {
      constexpr int LDA = LdsOperand<P, BM, BK>::LDK;
      constexpr int LDB = LdsOperand<P, BN, BK>::LDK;
      const float* A = reinterpret_cast<const float*>(sa);
      const float* B = reinterpret_cast<const float*>(sb);
#pragma unroll
      for (int kl = 0; kl < BK / 8 / WK; ++kl) {
        const int kc = kslice * (BK / 8 / WK) + kl;
        f32x4_t af[TM], bfr[TN];
#pragma unroll
        for (int i = 0; i < TM; ++i)
          af[i] = *reinterpret_cast<const f32x4_t*>(A + (wm_off + 32 * i + lr) * LDA + kc * 8 + lh * 4);
#pragma unroll
        for (int j = 0; j < TN; ++j)
          bfr[j] = *reinterpret_cast<const f32x4_t*>(B + (wn_off + 32 * j + lr) * LDB + kc * 8 + lh * 4);
        if (kl == 0) between(0);
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
          for (int i = 0; i < TM; ++i)
#pragma unroll
            for (int j = 0; j < TN; ++j)
              acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(af[i][q], bfr[j][q], acc[i][j], 0, 0, 0);
      }
    } else {
      constexpr int LDA = LdsOperand<P, BM, BK>::LDH;
      constexpr int LDB = LdsOperand<P, BN, BK>::LDH;
      constexpr int NPL = PrecInfo<P>::planes;
      const __bf16* A = reinterpret_cast<const __bf16*>(sa);
      const __bf16* B = reinterpret_cast<const __bf16*>(sb);
      // this wave's k-chunks of the stage: kslice * NKC + [0, NKC)
      constexpr int NKC = BK / 16 / WK;
      const int kc0 = kslice * NKC;
      auto fa = [&](int kc, int p, int i) {
        return *reinterpret_cast<const bf16x8_t*>(A + p * BM * LDA + bf16_slot<BK>(wm_off + 32 * i + lr, (kc0 + kc) * 16 + lh * 8));
      };
      auto fb = [&](int kc, int p, int j) {
        return *reinterpret_cast<const bf16x8_t*>(B + p * BN * LDB + bf16_slot<BK>(wn_off + 32 * j + lr, (kc0 + kc) * 16 + lh * 8));
      };
      if constexpr (P == P_BF16) {
        bf16x8_t af[NKC][TM], bfr[NKC][TN];
#pragma unroll
        for (int kc = 0; kc < NKC; ++kc) {
#pragma unroll
          for (int i = 0; i < TM; ++i) af[kc][i] = fa(kc, 0, i);
#pragma unroll
          for (int j = 0; j < TN; ++j) bfr[kc][j] = fb(kc, 0, j);
        }
        between(0);
#pragma unroll
        for (int kc = 0; kc < NKC; ++kc)
#pragma unroll
          for (int i = 0; i < TM; ++i)
#pragma unroll
            for (int j = 0; j < TN; ++j)
              acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(af[kc][i], bfr[kc][j], acc[i][j], 0, 0, 0);
      } else {
        // The term products are summed by the matrix cores into a temporary
        // that starts from zero every FLUSH stages and is then added to the
        // running accumulator with a round-to-nearest-even VALU add.
        // Repeated matrix-core accumulation onto a large running sum drifts
        // (measured bias of about -1e-6 relative at K = 2048); a small
        // temporary keeps that drift proportional to the temporary.
        // The fragments of the narrower side stay resident; the other side's
        // term planes are read one 32-wide block at a time.
        const f32x16_t zero = {};
        if constexpr (CHAIN) {
          // Wide wave tiles: each 32x32 block's term products over the whole
          // stage form one zero-based chain, added to the accumulator at its
          // end.  The narrower side's fragments stay resident.  Part b of
          // `between` is issued after block b's products, so its VALU and
          // LDS work overlaps the matrix cores.  The add is written as an FMA
          // with an opaque 1.0 (exact: rounds t + acc once, like the add) so
          // that the accumulator is updated in place; a plain add lets the
          // register allocator rotate accumulators between blocks and spill.
          float one;
          asm("v_mov_b32 %0, 1.0" : "=v"(one));
          if constexpr (TM >= TN) {
            bf16x8_t bfr[NKC][NPL][TN];
#pragma unroll
            for (int kc = 0; kc < NKC; ++kc)
#pragma unroll
              for (int p = 0; p < NPL; ++p)
#pragma unroll
                for (int j = 0; j < TN; ++j) bfr[kc][p][j] = fb(kc, p, j);
#pragma unroll
            for (int i = 0; i < TM; ++i) {
              f32x16_t t[TN];
#pragma unroll
              for (int kc = 0; kc < NKC; ++kc) {
                bf16x8_t af[NPL];
#pragma unroll
                for (int p = 0; p < NPL; ++p) af[p] = fa(kc, p, i);
#pragma unroll
                for (int j = 0; j < TN; ++j)
#pragma unroll
                  for (int q = 0; q < PrecInfo<P>::nprod; ++q)
                    t[j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(af[prod_a(P, q)], bfr[kc][prod_b(P, q)][j],
                                                                   (kc == 0 && q == 0) ? zero : t[j], 0, 0, 0);
              }
              between(i);
#pragma unroll
              for (int j = 0; j < TN; ++j)
#pragma unroll
                for (int r = 0; r < 16; ++r) acc[i][j][r] = __builtin_fmaf(t[j][r], one, acc[i][j][r]);
              __builtin_amdgcn_sched_barrier(0);
            }
          } else {
            bf16x8_t af[NKC][NPL][TM];
#pragma unroll
            for (int kc = 0; kc < NKC; ++kc)
#pragma unroll
              for (int p = 0; p < NPL; ++p)
#pragma unroll
                for (int i = 0; i < TM; ++i) af[kc][p][i] = fa(kc, p, i);
#pragma unroll
            for (int j = 0; j < TN; ++j) {
              f32x16_t t[TM];
#pragma unroll
              for (int kc = 0; kc < NKC; ++kc) {
                bf16x8_t bfr[NPL];
#pragma unroll
                for (int p = 0; p < NPL; ++p) bfr[p] = fb(kc, p, j);
#pragma unroll
                for (int i = 0; i < TM; ++i)
#pragma unroll
                  for (int q = 0; q < PrecInfo<P>::nprod; ++q)
                    t[i] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(af[kc][prod_a(P, q)][i], bfr[prod_b(P, q)],
                                                                   (kc == 0 && q == 0) ? zero : t[i], 0, 0, 0);
              }
              between(j);
#pragma unroll
              for (int i = 0; i < TM; ++i)
#pragma unroll
                for (int r = 0; r < 16; ++r) acc[i][j][r] = __builtin_fmaf(t[i][r], one, acc[i][j][r]);
              __builtin_amdgcn_sched_barrier(0);
            }
          }
        } else {
#pragma unroll
        for (int kc = 0; kc < NKC; ++kc) {
          if constexpr (TM * TN <= 4) {
            bf16x8_t af[NPL][TM], bfr[NPL][TN];
#pragma unroll
            for (int p = 0; p < NPL; ++p) {
#pragma unroll
              for (int i = 0; i < TM; ++i) af[p][i] = fa(kc, p, i);
#pragma unroll
              for (int j = 0; j < TN; ++j) bfr[p][j] = fb(kc, p, j);
            }
            if (kc == 0) between(0);
#pragma unroll
            for (int q = 0; q < PrecInfo<P>::nprod; ++q)
#pragma unroll
              for (int j = 0; j < TN; ++j)
#pragma unroll
                for (int i = 0; i < TM; ++i)
                  tmp[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(af[prod_a(P, q)][i], bfr[prod_b(P, q)][j],
                                                                      (first && kc == 0 && q == 0) ? zero : tmp[i][j], 0, 0, 0);
          } else if constexpr (TM >= TN) {
            bf16x8_t bfr[NPL][TN];
#pragma unroll
            for (int p = 0; p < NPL; ++p)
#pragma unroll
              for (int j = 0; j < TN; ++j) bfr[p][j] = fb(kc, p, j);
            if (kc == 0) between(0);
#pragma unroll
            for (int i = 0; i < TM; ++i) {
              bf16x8_t af[NPL];
#pragma unroll
              for (int p = 0; p < NPL; ++p) af[p] = fa(kc, p, i);
#pragma unroll
              for (int q = 0; q < PrecInfo<P>::nprod; ++q)
#pragma unroll
                for (int j = 0; j < TN; ++j)
                  tmp[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(af[prod_a(P, q)], bfr[prod_b(P, q)][j],
                                                                      (first && kc == 0 && q == 0) ? zero : tmp[i][j], 0, 0, 0);
            }
          } else {
            bf16x8_t af[NPL][TM];
#pragma unroll
            for (int p = 0; p < NPL; ++p)
#pragma unroll
              for (int i = 0; i < TM; ++i) af[p][i] = fa(kc, p, i);
            if (kc == 0) between(0);
#pragma unroll
            for (int j = 0; j < TN; ++j) {
              bf16x8_t bfr[NPL];
#pragma unroll
              for (int p = 0; p < NPL; ++p) bfr[p] = fb(kc, p, j);
#pragma unroll
              for (int q = 0; q < PrecInfo<P>::nprod; ++q)
#pragma unroll
                for (int i = 0; i < TM; ++i)
                  tmp[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(af[prod_a(P, q)][i], bfr[prod_b(P, q)],
                                                                      (first && kc == 0 && q == 0) ? zero : tmp[i][j], 0, 0, 0);
            }
          }
        }
        if (flush) flush_tmp(acc, tmp);
        }
      }
    }
  }

  // gk_lds: a copy of d.gk in LDS (the per-stage offset loop indexes it dynamically)
  __device__ static __forceinline__ void run(const GemmDesc& d, const Group& gk_lds, int bid, int bz, char* smem) {
    int tm, tn;
    tile_coords(bid, d.tiles_m, d.tiles_n, tm, tn);
    const int wave = threadIdx.x >> 6;
    const int wmn = wave % (WM * WN);
    const int kslice = WK > 1 ? __builtin_amdgcn_readfirstlane(wave / (WM * WN)) : 0;
    const int wm_off = (wmn % WM) * (BM / WM);
    const int wn_off = (wmn / WM) * (BN / WN);
    const int m0 = tm * BM, n0 = tn * BN;

    float scale = 1.0f;
    if (d.a_scale_bits) scale = pow2_inverse_scale(d.a_scale_bits[bz]);

    f32x16_t acc[TM][TN];
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
      for (int j = 0; j < TN; ++j)
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.f;
    f32x16_t tmp[TMT][TNT];

    const int nk = (d.K + BK - 1) / BK;
    if constexpr (AMODE < 0 || BMODE < 0) {
      OperandLoader<P, BM, BK, NT, 0> la;
      OperandLoader<P, BN, BK, NT, 1> lb;
      la.init(d.a_mode, d.a + bz * d.a_bs, d.gm, m0, d.M, d.K, 1.0f);
      lb.init(d.b_mode, d.b + bz * d.b_bs, d.gn, n0, d.N, d.K, 1.0f);
      la.load(0, gk_lds);
      lb.load(0, gk_lds);
      la.store(smem);
      lb.store(smem + bytesA);
      __syncthreads();
      // stages in groups of FLUSH, unrolled so the temporary's first and last
      // stage are known at compile time
      for (int kt0 = 0; kt0 < nk; kt0 += FLUSH) {
#pragma unroll
        for (int s = 0; s < FLUSH; ++s) {
          const int kt = kt0 + s;
          if (kt < nk) {
            char* cur = smem + (kt & 1) * stage;
            char* nxt = smem + ((kt + 1) & 1) * stage;
            const bool more = kt + 1 < nk;
            if (more) {
              la.load((kt + 1) * BK, gk_lds);
              lb.load((kt + 1) * BK, gk_lds);
            }
            compute(cur, cur + bytesA, acc, tmp, s == 0, s == FLUSH - 1, wm_off, wn_off, kslice);
            if (more) {
              la.store(nxt);
              lb.store(nxt + bytesA);
            }
            __syncthreads();
          }
        }
      }
      if (nk % FLUSH != 0) flush_tmp(acc, tmp);
    } else {
      FastLoader<P, BM, BK, NT, AMODE, DEPTH> la;
      FastLoader<P, BN, BK, NT, BMODE, DEPTH> lb;
      la.init(d.a + bz * d.a_bs, d.gm, m0, d.M, d.gk.s[0][0], d.K);
      lb.init(d.b + bz * d.b_bs, d.gn, n0, d.N, d.gk.s[1][0], d.K);
      using LA = FastLoader<P, BM, BK, NT, AMODE, DEPTH>;
      using LB = FastLoader<P, BN, BK, NT, BMODE, DEPTH>;
      constexpr int NVA = LA::NV, NVB = LB::NV;
      // load slots (A's, then B's) spread evenly over the parts of `between`
      auto part_of = [](int v) { return v * NPARTS / (NVA + NVB); };
      // Software pipeline: global loads run ahead in DEPTH register sets
      // (set = stage parity when DEPTH = 2; with one set it is refilled right
      // after its stage is stored); while stage kt's MFMAs run, stage kt+1
      // is split and stored into the other LDS buffer.  One barrier per stage.
      la.template load_stage<0>(0, nk);
      lb.template load_stage<0>(0, nk);
      if constexpr (DEPTH == 2) {
        la.template load_stage<1>(1, nk);
        lb.template load_stage<1>(1, nk);
      }
      la.template store<0>(smem);
      lb.template store<0>(smem + bytesA);
      if constexpr (DEPTH == 1) {
        // one register set: it is refilled as soon as its stage is stored
        la.template load_stage<0>(1, nk);
        lb.template load_stage<0>(1, nk);
      }
      __syncthreads();
      static_assert(FLUSH % 2 == 0 || FLUSH == 1, "stage groups must keep the register-set parity static");
      constexpr int G = FLUSH == 1 ? 2 : FLUSH;   // stages per unrolled group (even)
      // how far ahead of the computed stage the last issued load runs
      constexpr int AHEAD = DEPTH == 1 ? 2 : DEPTH;
      int kt0 = 0;
      // steady state: every stage of the group loads a full stage AHEAD
      // stages on and stores the next one, so a stage is one straight-line
      // block that the scheduler can interleave (loads, split, LDS traffic
      // and MFMAs)
      // (the last stage, which holds k = K - 1, is loaded in the tail loop)
      for (; kt0 + G - 1 + AHEAD < nk - 1; kt0 += G) {
#pragma unroll
        for (int s = 0; s < G; ++s) {
          const int kt = kt0 + s;
          char* cur = smem + (s & 1) * stage;
          char* nxt = smem + ((s + 1) & 1) * stage;
          const bool first = FLUSH == 1 ? true : s == 0;
          const bool flush = FLUSH == 1 ? true : s == FLUSH - 1;
          if constexpr (DEPTH == 1) {
            // each slot of stage kt+1 (in registers since the same part of
            // stage kt-1) goes to LDS, then its registers take stage kt+2:
            // every load has a whole stage of matrix-core work to arrive
            auto st_next = [&](int part) {
#pragma unroll
              for (int v = 0; v < NVA + NVB; ++v)
                if (part_of(v) == part) {
                  if (v < NVA) {
                    la.template store_slot<0>(nxt, v);
                    la.template load_slot<false, 0>((kt + 2) * BK, v);
                  } else {
                    lb.template store_slot<0>(nxt + bytesA, v - NVA);
                    lb.template load_slot<false, 0>((kt + 2) * BK, v - NVA);
                  }
                }
            };
            compute(cur, cur + bytesA, acc, tmp, first, flush, wm_off, wn_off, kslice, st_next);
          } else if (s & 1) {
            la.template load<false, 1>((kt + 2) * BK);
            lb.template load<false, 1>((kt + 2) * BK);
            auto st_next = [&](int part) {
#pragma unroll
              for (int v = 0; v < NVA + NVB; ++v)
                if (part_of(v) == part) {
                  if (v < NVA)
                    la.template store_slot<0>(nxt, v);
                  else
                    lb.template store_slot<0>(nxt + bytesA, v - NVA);
                }
            };
            compute(cur, cur + bytesA, acc, tmp, first, flush, wm_off, wn_off, kslice, st_next);
          } else {
            la.template load<false, 0>((kt + 2) * BK);
            lb.template load<false, 0>((kt + 2) * BK);
            auto st_next = [&](int part) {
#pragma unroll
              for (int v = 0; v < NVA + NVB; ++v)
                if (part_of(v) == part) {
                  if (v < NVA)
                    la.template store_slot<1>(nxt, v);
                  else
                    lb.template store_slot<1>(nxt + bytesA, v - NVA);
                }
            };
            compute(cur, cur + bytesA, acc, tmp, first, flush, wm_off, wn_off, kslice, st_next);
          }
          __syncthreads();
        }
      }
      // the last groups: loads may be partial or absent
      for (; kt0 < nk; kt0 += G) {
#pragma unroll
        for (int s = 0; s < G; ++s) {
          const int kt = kt0 + s;
          if (kt < nk) {
            char* cur = smem + (s & 1) * stage;
            char* nxt = smem + ((s + 1) & 1) * stage;
            const bool first = FLUSH == 1 ? true : s == 0;
            const bool flush = FLUSH == 1 ? true : s == FLUSH - 1;
            if constexpr (DEPTH == 1) {
              auto st_next = [&](int part) {
                if (part != 0) return;
                if (kt + 1 < nk) {
                  la.template store<0>(nxt);
                  lb.template store<0>(nxt + bytesA);
                }
                la.template load_stage<0>(kt + 2, nk);
                lb.template load_stage<0>(kt + 2, nk);
              };
              compute(cur, cur + bytesA, acc, tmp, first, flush, wm_off, wn_off, kslice, st_next);
            } else if (s & 1) {
              la.template load_stage<1>(kt + 2, nk);
              lb.template load_stage<1>(kt + 2, nk);
              auto st_next = [&](int part) {
                if (part == 0 && kt + 1 < nk) {
                  la.template store<0>(nxt);
                  lb.template store<0>(nxt + bytesA);
                }
              };
              compute(cur, cur + bytesA, acc, tmp, first, flush, wm_off, wn_off, kslice, st_next);
            } else {
              la.template load_stage<0>(kt + 2, nk);
              lb.template load_stage<0>(kt + 2, nk);
              auto st_next = [&](int part) {
                if (part == 0 && kt + 1 < nk) {
                  la.template store<1>(nxt);
                  lb.template store<1>(nxt + bytesA);
                }
              };
              compute(cur, cur + bytesA, acc, tmp, first, flush, wm_off, wn_off, kslice, st_next);
            }
            __syncthreads();
          }
        }
      }
      if (nk % FLUSH != 0) flush_tmp(acc, tmp);
    }

    if constexpr (WK > 1) {
      // add the k-slice groups' sums into group 0 through LDS (free after
      // the last stage): lane-contiguous rows of [wave][block][register]
      float* red = reinterpret_cast<float*>(smem);
      const int lane = threadIdx.x & 63;
#pragma unroll 1
      for (int g = 1; g < WK; ++g) {
        __syncthreads();
        if (kslice == g) {
#pragma unroll
          for (int i = 0; i < TM; ++i)
#pragma unroll
            for (int j = 0; j < TN; ++j)
#pragma unroll
              for (int r = 0; r < 16; ++r) red[((wmn * TM * TN + i * TN + j) * 16 + r) * 64 + lane] = acc[i][j][r];
        }
        __syncthreads();
        if (kslice == 0) {
#pragma unroll
          for (int i = 0; i < TM; ++i)
#pragma unroll
            for (int j = 0; j < TN; ++j)
#pragma unroll
              for (int r = 0; r < 16; ++r) acc[i][j][r] += red[((wmn * TM * TN + i * TN + j) * 16 + r) * 64 + lane];
        }
      }
      __syncthreads();
    }

    // epilogue.  The output offsets of the tile's BM rows and BN columns are
    // formed once into LDS (free after the last stage), so the store loop is
    // a short fully-unrolled sequence.  C layout of a 32x32 block: lane l,
    // register r holds row 8*(r/4) + 4*(l/32) + r%4, column l%32.
    static_assert((BM + BN) * 8 <= lds_bytes, "LDS too small for the offset tables");
    int64_t* offm = reinterpret_cast<int64_t*>(smem);
    int64_t* offn = offm + BM;
    for (int e = threadIdx.x; e < BM + BN; e += NT) {
      int64_t o[1] = {0};
      if (e < BM) {
        if (m0 + e < d.M) group_offsets<1>(d.gm, (uint32_t)(m0 + e), o, 1);
        offm[e] = o[0];
      } else {
        if (n0 + e - BM < d.N) group_offsets<1>(d.gn, (uint32_t)(n0 + e - BM), o, 1);
        offn[e - BM] = o[0];
      }
    }
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const int lr = lane & 31, lh = lane >> 5;
    float* C = d.c + bz * d.c_bs;
    float amax = 0.f;
    const bool mvec = d.c_mode == STORE_MVEC;
    // the operand rescale 2^-e (exact) is applied to the product instead of the A operand
    const bool scaled = scale != 1.0f;
    // with k-slice groups only group 0 holds the sums
    if (WK == 1 || kslice == 0) {
#pragma unroll
    for (int j = 0; j < TN; ++j) {
      const int nl = wn_off + 32 * j + lr;
      const bool nok = n0 + nl < d.N;
      const int64_t on = offn[nl];
#pragma unroll
      for (int i = 0; i < TM; ++i) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int ml = wm_off + 32 * i + 8 * q + 4 * lh;
          f32x4_t v = {acc[i][j][4 * q + 0], acc[i][j][4 * q + 1], acc[i][j][4 * q + 2], acc[i][j][4 * q + 3]};
          if (scaled) v *= scale;
          if (nok && m0 + ml < d.M) {
            if (mvec) {
              *reinterpret_cast<f32x4_t*>(C + offm[ml] + on) = v;
#pragma unroll
              for (int r = 0; r < 4; ++r) amax = fmaxf(amax, fabsf(v[r]));
            } else {
#pragma unroll
              for (int r = 0; r < 4; ++r)
                if (m0 + ml + r < d.M) {
                  C[offm[ml + r] + on] = v[r];
                  amax = fmaxf(amax, fabsf(v[r]));
                }
            }
          }
        }
      }
    }
    }
    if (d.c_absmax) {
#pragma unroll
      for (int o = 32; o >= 1; o >>= 1) amax = fmaxf(amax, __shfl_xor(amax, o, 64));
      if (lane == 0) atomicMax(d.c_absmax + bz, __float_as_uint(amax));
    }
  }
};

}  // namespace tn
