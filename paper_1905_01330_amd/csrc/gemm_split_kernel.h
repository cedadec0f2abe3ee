// Split-BF16 contraction kernel with a lean stage (gfx950, CDNA4).
//
// The same product as the general tile kernel in gemm_kernel.h,
// C[m, n] = sum_k A[m, k] B[k, n] with every FP32 operand split into three
// BF16 terms and six term products per k-step, specialised for the layouts
// of the large contractions: A read along k (one merged contracted axis of
// unit stride) and B read along k, or element by element along k with the
// lanes along n.  The index groups of M and N stay arbitrary (row offsets
// come from the group descriptors), so the permutation is still fused into
// the loads.
//
// What differs from the general kernel, all to cut the vector-ALU work per
// stage (there about 450 vector instructions per wave against 60 matrix-core
// products):
//   * buffer loads with the operand base in scalar registers: the per-stage
//     advance is a scalar offset, so the loads cost no vector address math;
//   * every thread moves whole 8-k runs of one row (two 16-byte loads when k
//     is contiguous, eight 4-byte loads along k when n is: the lanes of a
//     wavefront then read 64 consecutive n, and no register transpose is
//     needed), and writes each BF16 term plane with one 16-byte LDS store;
//   * the split and the LDS stores are spread over the stage between the
//     products of consecutive block rows.
// The term products of a block over one stage form a zero-based chain that
// is added to the accumulator with a vector add, as in the general kernel.
#pragma once

#include <type_traits>

#include "gemm_kernel.h"

namespace tn {

typedef uint32_t u32x4_t __attribute__((ext_vector_type(4)));

__device__ __forceinline__ __amdgpu_buffer_rsrc_t split_rsrc(const float* p) {
  // raw buffer (stride 0) over the whole 32-bit offset range; the host
  // checks that every offset of the view fits
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(p), (short)0, (int)0xffffffff, 0x00020000);
}

// BM x BN tile, BK = 32 per stage, WN waves side by side (each wave owns a
// BM x BN/WN column strip of TM x TN blocks of 32 x 32), both operands split
// into LDS (two stage buffers).  BMODE: LOAD_KVEC (B k-contiguous, 16-byte
// loads) or LOAD_MNVEC (one element per lane along k, the lanes along n: any
// B layout with a single contracted axis).
template <int BM, int BN, int WN, int BMODE>
struct SplitGemm {
  static constexpr int BK = 32;
  static constexpr int NW = WN;
  static constexpr int NT = NW * 64;
  static constexpr int TM = BM / 32;
  static constexpr int TN = BN / WN / 32;
  static constexpr int CH = BK / 8;        // 8-k runs per row and stage
  static constexpr int NKC = BK / 16;      // matrix-core k-steps per stage
  static constexpr int NA = BM * CH;       // A runs per stage
  static constexpr int NB = BN * CH;       // B runs per stage
  static constexpr int NSLOT = (NA + NB + NT - 1) / NT;
  static constexpr int PA = BM * BK;       // BF16 elements per A plane
  static constexpr int PB = BN * BK;
  static constexpr int bytesA = 3 * PA * 2;
  static constexpr int bytesB = 3 * PB * 2;
  static constexpr int stage = bytesA + bytesB;
  static constexpr int lds_bytes = 2 * stage;
  __device__ static constexpr int stage_bytes() { return stage; }
  static_assert(BM % 32 == 0 && BN % 64 == 0 && TN >= 1 && TN * WN * 32 == BN, "tile shape");
  static_assert(NA % 64 == 0 && NB % 64 == 0 && NT % 64 == 0, "every wavefront's run of a slot is one operand");
  static_assert(lds_bytes <= 160 * 1024, "LDS");

  // run r of a stage: (operand, row, 8-k chunk).  Sixteen consecutive runs
  // are sixteen consecutive rows with one chunk, so the 16-byte LDS stores of
  // a quarter wavefront hit distinct banks under bf16_slot.  A (and a
  // k-contiguous B) cycles the chunks every 16 rows, so a wavefront reads 16
  // whole 128-byte row segments; an n-contiguous B keeps 64 consecutive n
  // per wavefront and chunk, so each 4-byte load is one 256-byte run.
  __device__ static __forceinline__ void run_of(int r, bool& isb, int& row, int& chunk) {
    isb = r >= NA;
    const int q = isb ? r - NA : r;
    if (!isb || BMODE == LOAD_KVEC) {
      const int g = q >> 4;
      chunk = g % CH;
      row = (g / CH) * 16 + (q & 15);
    } else {
      chunk = (q >> 6) % CH;
      row = (q / (64 * CH)) * 64 + (q & 63);
    }
  }

  struct Slot {
    float x[8];
  };

  __device__ static __forceinline__ void run(const GemmDesc& d, int bid, int bz, char* smem) {
    int tm, tn;
    tile_coords(bid, d.tiles_m, d.tiles_n, tm, tn);
    const int tid = threadIdx.x;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int lane = tid & 63;
    const int lr = lane & 31, lh = lane >> 5;
    const int m0 = tm * BM, n0 = tn * BN;
    const int wn_off = wave * (TN * 32);

    float scale = 1.0f;
    if (d.a_scale_bits) scale = pow2_inverse_scale(d.a_scale_bits[bz]);

    const __amdgpu_buffer_rsrc_t ra = split_rsrc(d.a + bz * d.a_bs);
    const __amdgpu_buffer_rsrc_t rb = split_rsrc(d.b + bz * d.b_bs);
    const int K = d.K;
    const int sbk = (int)d.gk.s[1][0];   // B's stride along k (elements); 1 when k-contiguous

    // per-slot global byte offset (stage 0) and LDS byte offset of the run
    uint32_t goff[NSLOT], loff[NSLOT];
#pragma unroll
    for (int v = 0; v < NSLOT; ++v) {
      const int r = v * NT + tid;
      bool isb;
      int row, chunk;
      run_of(r < NA + NB ? r : 0, isb, row, chunk);
      int64_t o[1];
      if (!isb) {
        int m = m0 + row;
        m = m < d.M ? m : d.M - 1;
        group_offsets<1>(d.gm, (uint32_t)m, o, 0);
        goff[v] = (uint32_t)((o[0] + chunk * 8) * 4);
        loff[v] = (uint32_t)(bf16_slot<BK>(row, chunk * 8) * 2);
      } else {
        int n = n0 + row;
        n = n < d.N ? n : d.N - 1;
        group_offsets<1>(d.gn, (uint32_t)n, o, 0);
        goff[v] = (uint32_t)((o[0] + (int64_t)chunk * 8 * sbk) * 4);
        loff[v] = (uint32_t)(bytesA + bf16_slot<BK>(row, chunk * 8) * 2);
      }
    }

    Slot sl[NSLOT];
    // slot v of stage kt (its kind is uniform over the wavefront); TAIL:
    // runs past K read as zeros
    auto load_slot = [&](int v, int kt, auto tail) {
      constexpr bool TAIL = decltype(tail)::value;
      const int r0 = v * NT + wave * 64;
      if (r0 >= NA + NB) return;
      const bool isb = r0 >= NA;
      const int k0 = kt * BK;
      bool ok = true;
      if constexpr (TAIL) {
        bool isb_;
        int row_, chunk_;
        run_of(v * NT + tid, isb_, row_, chunk_);
        ok = k0 + chunk_ * 8 < K;
      }
      if (!isb || BMODE == LOAD_KVEC) {
        const __amdgpu_buffer_rsrc_t rs = isb ? rb : ra;
        f32x4_t lo, hi;
        if constexpr (TAIL) {
          lo = f32x4_t{0.f, 0.f, 0.f, 0.f};
          hi = lo;
          if (ok) {
            lo = __builtin_bit_cast(f32x4_t, __builtin_amdgcn_raw_buffer_load_b128(rs, goff[v], k0 * 4, 0));
            hi = __builtin_bit_cast(f32x4_t, __builtin_amdgcn_raw_buffer_load_b128(rs, goff[v] + 16, k0 * 4, 0));
          }
        } else {
          lo = __builtin_bit_cast(f32x4_t, __builtin_amdgcn_raw_buffer_load_b128(rs, goff[v], k0 * 4, 0));
          hi = __builtin_bit_cast(f32x4_t, __builtin_amdgcn_raw_buffer_load_b128(rs, goff[v] + 16, k0 * 4, 0));
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          sl[v].x[j] = lo[j];
          sl[v].x[4 + j] = hi[j];
        }
      } else {
        const int sb = k0 * sbk * 4;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          if constexpr (TAIL) {
            float y = 0.f;
            if (ok) y = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rb, goff[v], sb + j * sbk * 4, 0));
            sl[v].x[j] = y;
          } else {
            sl[v].x[j] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rb, goff[v], sb + j * sbk * 4, 0));
          }
        }
      }
    };
    auto store_slot = [&](int v, char* buf) {
      const int r0 = v * NT + wave * 64;
      if (r0 >= NA + NB) return;
      const int pl = r0 >= NA ? PB * 2 : PA * 2;
      u32x4_t t0, t1, t2;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        uint32_t w[3];
        split_pair<3>(sl[v].x[2 * q], sl[v].x[2 * q + 1], w);
        t0[q] = w[0];
        t1[q] = w[1];
        t2[q] = w[2];
      }
      char* p = buf + loff[v];
      *reinterpret_cast<u32x4_t*>(p) = t0;
      *reinterpret_cast<u32x4_t*>(p + pl) = t1;
      *reinterpret_cast<u32x4_t*>(p + 2 * pl) = t2;
    };

    f32x16_t acc[TM][TN];
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
      for (int j = 0; j < TN; ++j)
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.f;
    // the flush below is an FMA with an opaque 1.0 (exact: it rounds t + acc
    // once, like an add) so that each accumulator is updated in place
    float one;
    asm("v_mov_b32 %0, 1.0" : "=v"(one));
    const f32x16_t zero = {};

    const int nk = (K + BK - 1) / BK;
    const int nfull = K / BK;

    // fragment addresses (bytes) of k-step kc within a stage: row lr of the
    // lane's 32-row block, k = kc * 16 + lh * 8
    uint32_t fa_off[NKC], fb_off[NKC];
#pragma unroll
    for (int kc = 0; kc < NKC; ++kc) {
      fa_off[kc] = (uint32_t)(bf16_slot<BK>(lr, kc * 16 + lh * 8) * 2);
      fb_off[kc] = (uint32_t)(bytesA + bf16_slot<BK>(wn_off + lr, kc * 16 + lh * 8) * 2);
    }

    using T_ = std::integral_constant<bool, true>;
    using F_ = std::integral_constant<bool, false>;
    // prologue: stage 0 into LDS buffer 0, stage 1 into registers
    if (nfull >= 1) {
#pragma unroll
      for (int v = 0; v < NSLOT; ++v) load_slot(v, 0, F_());
    } else {
#pragma unroll
      for (int v = 0; v < NSLOT; ++v) load_slot(v, 0, T_());
    }
#pragma unroll
    for (int v = 0; v < NSLOT; ++v) store_slot(v, smem);
    if (nfull >= 2) {
#pragma unroll
      for (int v = 0; v < NSLOT; ++v) load_slot(v, 1, F_());
    } else if (nk > 1) {
#pragma unroll
      for (int v = 0; v < NSLOT; ++v) load_slot(v, 1, T_());
    }
    __syncthreads();

    // One stage: the block rows i, each over the stage's k-steps, the A
    // fragments of the next step read before the current step's products
    // are issued.  A block's products of the stage form one chain on the
    // matrix cores that starts from zero (smallest products first); the
    // chain is added to the accumulator with one vector add (round to
    // nearest even), so the running sums never take a matrix-core
    // accumulation, whose rounding onto a large value drifts.  The next
    // stage's runs (in registers) are split and stored after steps spread
    // over the stage, and each slot's registers then take the loads of the
    // stage after.
    constexpr int NSTEP = NKC * TM;
    auto stage = [&](int kt, auto st, auto ld, auto tail) {
      constexpr bool ST = decltype(st)::value, LD = decltype(ld)::value;
      const char* cur = smem + (kt & 1) * stage_bytes();
      char* nxt = smem + ((kt + 1) & 1) * stage_bytes();
      // fragments: B of every k-step of the stage; A of the current step,
      // read one step ahead (two sets)
      bf16x8_t bf[NKC][TN][3], af[2][3];
#pragma unroll
      for (int kc = 0; kc < NKC; ++kc)
#pragma unroll
        for (int j = 0; j < TN; ++j)
#pragma unroll
          for (int p = 0; p < 3; ++p)
            bf[kc][j][p] = *reinterpret_cast<const bf16x8_t*>(cur + fb_off[kc] + p * PB * 2 + j * 32 * BK * 2);
      auto read_a = [&](int kc, int i, int set) {
#pragma unroll
        for (int p = 0; p < 3; ++p)
          af[set][p] = *reinterpret_cast<const bf16x8_t*>(cur + fa_off[kc] + p * PA * 2 + i * 32 * BK * 2);
      };
      read_a(0, 0, 0);
      f32x16_t ch[TN];
#pragma unroll
      for (int s = 0; s < NSTEP; ++s) {
        const int i = s / NKC, kc = s % NKC;
        const int sa = s & 1;
        if (s + 1 < NSTEP) read_a((s + 1) % NKC, (s + 1) / NKC, sa ^ 1);
        // consecutive products go to different blocks when TN > 1
#pragma unroll
        for (int q = 0; q < 6; ++q)
#pragma unroll
          for (int j = 0; j < TN; ++j) {
            const int pa = q == 0 ? 1 : q == 1 ? 0 : q == 2 ? 2 : q == 3 ? 0 : q == 4 ? 1 : 0;
            const int pb = q == 0 ? 1 : q == 1 ? 2 : q == 2 ? 0 : q == 3 ? 1 : q == 4 ? 0 : 0;
            ch[j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(af[sa][pa], bf[kc][j][pb],
                                                            (kc == 0 && q == 0) ? zero : ch[j], 0, 0, 0);
          }
        if (kc == NKC - 1) {
#pragma unroll
          for (int j = 0; j < TN; ++j)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[i][j][r] = __builtin_fmaf(ch[j][r], one, acc[i][j][r]);
        }
#pragma unroll
        for (int v = 0; v < NSLOT; ++v)
          if ((v * NSTEP) / NSLOT == s) {
            if constexpr (ST) store_slot(v, nxt);
            if constexpr (LD) load_slot(v, kt + 2, tail);
          }
      }
      __syncthreads();
    };

    // steady state: every stage stores the next one and loads a full stage;
    // then at most three stages remain (K % BK != 0 adds a partial one)
    int kt = 0;
    for (; kt + 2 < nfull; ++kt) stage(kt, T_(), T_(), F_());
    if (kt + 2 < nk) {
      stage(kt, T_(), T_(), T_());
      ++kt;
    }
    if (kt + 1 < nk) {
      stage(kt, T_(), F_(), F_());
      ++kt;
    }
    if (kt < nk) stage(kt, F_(), F_(), F_());

    static_assert((BM + BN) * 8 <= lds_bytes, "LDS too small for the offset tables");
    int64_t* offm = reinterpret_cast<int64_t*>(smem);
    int64_t* offn = offm + BM;
    for (int e = tid; e < BM + BN; e += NT) {
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
    float* C = d.c + bz * d.c_bs;
    float amax = 0.f;
    const bool mvec = d.c_mode == STORE_MVEC;
    const bool scaled = scale != 1.0f;
#pragma unroll
    for (int j = 0; j < TN; ++j) {
      const int nl = wn_off + 32 * j + lr;
      const bool nok = n0 + nl < d.N;
      const int64_t on = offn[nl];
#pragma unroll
      for (int i = 0; i < TM; ++i) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int ml = 32 * i + 8 * q + 4 * lh;
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
    if (d.c_absmax) {
#pragma unroll
      for (int o = 32; o >= 1; o >>= 1) amax = fmaxf(amax, __shfl_xor(amax, o, 64));
      if (lane == 0) atomicMax(d.c_absmax + bz, __float_as_uint(amax));
    }
  }
};

// BM x BN tile, BK = 32 per stage, BN / 32 waves side by side, each owning a
// BM x 32 column strip of TM blocks; with WK = 2 there are two such groups
// of waves, each taking one of the stage's two k-steps, and their sums are
// added through LDS at the end.  Only A, which every wave reads,
// passes through LDS (three stage buffers, written two stages ahead); each
// wave's own 32 columns of B go from global memory straight to its
// registers, are split there and are used as the matrix-core operand as
// they are.  Three buffers let a wave read the next stage's first A
// fragments before the stage barrier, so the barrier does not drain the
// matrix cores.  BMODE as for SplitGemm.
template <int BM, int BN, int BMODE, int WK>
struct SplitGemmP {
  static constexpr int BK = 32;
  static constexpr int NWC = BN / 32;      // waves along N
  static constexpr int NW = NWC * WK;
  static constexpr int NT = NW * 64;
  static constexpr int TM = BM / 32;
  static constexpr int CH = BK / 8;        // 8-k runs per row and stage
  static constexpr int NKC = BK / 16;      // matrix-core k-steps per stage
  static constexpr int KPG = NKC / WK;     // k-steps per wave group
  static constexpr int NA = BM * CH;       // A runs per stage
  static constexpr int RPW = NA / NW;      // A runs per wave and stage
  static constexpr int NSA = (RPW + 63) / 64;
  static constexpr int PA = BM * BK;       // BF16 elements per A plane
  static constexpr int stage = 3 * PA * 2;
  static constexpr int NBUF = 3;
  static constexpr int lds_bytes = NBUF * stage;
  static_assert(BM % 32 == 0 && BN % 32 == 0, "tile shape");
  static_assert(NA % NW == 0 && RPW % 16 == 0, "each wave stores whole 16-row groups");
  static_assert(lds_bytes <= 160 * 1024 && (BM + BN) * 8 <= lds_bytes, "LDS");
  static_assert(NKC % WK == 0 && (WK == 1 || NWC * TM * 16 * 64 * 4 <= lds_bytes), "k groups");

  __device__ static __forceinline__ void run(const GemmDesc& d, int bid, int bz, char* smem) {
    int tm, tn;
    tile_coords(bid, d.tiles_m, d.tiles_n, tm, tn);
    const int tid = threadIdx.x;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int lane = tid & 63;
    const int lr = lane & 31, lh = lane >> 5;
    const int m0 = tm * BM, n0 = tn * BN;
    const int kg = WK > 1 ? __builtin_amdgcn_readfirstlane(wave / NWC) : 0;   // k group
    const int wn_off = (wave % NWC) * 32;

    float scale = 1.0f;
    if (d.a_scale_bits) scale = pow2_inverse_scale(d.a_scale_bits[bz]);

    const __amdgpu_buffer_rsrc_t ra = split_rsrc(d.a + bz * d.a_bs);
    const __amdgpu_buffer_rsrc_t rb = split_rsrc(d.b + bz * d.b_bs);
    const int K = d.K;
    const int sbk = (int)d.gk.s[1][0];   // B's stride along k (elements)
    const int nk = (K + BK - 1) / BK;
    const int nfull = K / BK;

    // ---- A runs: wave w stores runs [w * RPW, (w + 1) * RPW) of a stage;
    // sixteen consecutive runs are sixteen consecutive rows with one 8-k chunk
    uint32_t agoff[NSA], aloff[NSA];
#pragma unroll
    for (int v = 0; v < NSA; ++v) {
      const int r = wave * RPW + v * 64 + (lane < RPW - v * 64 ? lane : 0);
      const int g = r >> 4;
      const int chunk = g % CH;
      const int row = (g / CH) * 16 + (r & 15);
      int m = m0 + row;
      m = m < d.M ? m : d.M - 1;
      int64_t o[1];
      group_offsets<1>(d.gm, (uint32_t)m, o, 0);
      agoff[v] = (uint32_t)((o[0] + chunk * 8) * 4);
      aloff[v] = (uint32_t)(bf16_slot<BK>(row, chunk * 8) * 2);
    }
    float ax[NSA][8];
    auto a_load = [&](int v, int kt, bool tail) {
      const int k0 = kt * BK;
      f32x4_t lo = {0.f, 0.f, 0.f, 0.f}, hi = lo;
      // the run's 8-k chunk (only the last, partial stage needs it)
      if (!tail || k0 + ((((wave * RPW + v * 64 + (lane < RPW - v * 64 ? lane : 0)) >> 4) % CH) * 8) < K) {
        lo = __builtin_bit_cast(f32x4_t, __builtin_amdgcn_raw_buffer_load_b128(ra, agoff[v], k0 * 4, 0));
        hi = __builtin_bit_cast(f32x4_t, __builtin_amdgcn_raw_buffer_load_b128(ra, agoff[v] + 16, k0 * 4, 0));
      }
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        ax[v][j] = lo[j];
        ax[v][4 + j] = hi[j];
      }
    };
    auto a_store = [&](int v, char* buf) {
      if (v * 64 + 64 > RPW && lane >= RPW - v * 64) return;
      u32x4_t t0, t1, t2;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        uint32_t w[3];
        split_pair<3>(ax[v][2 * q], ax[v][2 * q + 1], w);
        t0[q] = w[0];
        t1[q] = w[1];
        t2[q] = w[2];
      }
      char* p = buf + aloff[v];
      *reinterpret_cast<u32x4_t*>(p) = t0;
      *reinterpret_cast<u32x4_t*>(p + PA * 2) = t1;
      *reinterpret_cast<u32x4_t*>(p + 2 * PA * 2) = t2;
    };

    // ---- B: lane (lr, lh) holds column n0 + wn_off + lr, k = 16 kc + 8 lh + 0..7
    // for the group's k-steps kc = kg * KPG + lk
    uint32_t bgoff;
    {
      int n = n0 + wn_off + lr;
      n = n < d.N ? n : d.N - 1;
      int64_t o[1];
      group_offsets<1>(d.gn, (uint32_t)n, o, 0);
      bgoff = (uint32_t)((o[0] + (int64_t)(8 * lh) * sbk) * 4);
    }
    float bx[KPG][8];
    auto b_load = [&](int kc, int kt, bool tail) {
      const int k0 = kt * BK + (kg * KPG + kc) * 16;
      const bool ok = !tail || k0 + 8 * lh < K;
      if (BMODE == LOAD_KVEC) {
        f32x4_t lo = {0.f, 0.f, 0.f, 0.f}, hi = lo;
        if (ok) {
          lo = __builtin_bit_cast(f32x4_t, __builtin_amdgcn_raw_buffer_load_b128(rb, bgoff, k0 * 4, 0));
          hi = __builtin_bit_cast(f32x4_t, __builtin_amdgcn_raw_buffer_load_b128(rb, bgoff + 16, k0 * 4, 0));
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          bx[kc][j] = lo[j];
          bx[kc][4 + j] = hi[j];
        }
      } else {
        const int sb = k0 * sbk * 4;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          float y = 0.f;
          if (ok) y = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rb, bgoff, sb + j * sbk * 4, 0));
          bx[kc][j] = y;
        }
      }
    };
    bf16x8_t bf[KPG][3];
    auto b_split = [&](int kc) {
      u32x4_t t0, t1, t2;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        uint32_t w[3];
        split_pair<3>(bx[kc][2 * q], bx[kc][2 * q + 1], w);
        t0[q] = w[0];
        t1[q] = w[1];
        t2[q] = w[2];
      }
      bf[kc][0] = __builtin_bit_cast(bf16x8_t, t0);
      bf[kc][1] = __builtin_bit_cast(bf16x8_t, t1);
      bf[kc][2] = __builtin_bit_cast(bf16x8_t, t2);
    };

    f32x16_t acc[TM];
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[i][r] = 0.f;

    uint32_t fa_off[KPG];
#pragma unroll
    for (int kc = 0; kc < KPG; ++kc) fa_off[kc] = (uint32_t)(bf16_slot<BK>(lr, (kg * KPG + kc) * 16 + lh * 8) * 2);
    bf16x8_t af[2][3];   // A fragments, read one step ahead
    auto read_a = [&](const char* buf, int kc, int i, int set) {
#pragma unroll
      for (int p = 0; p < 3; ++p)
        af[set][p] = *reinterpret_cast<const bf16x8_t*>(buf + fa_off[kc] + p * PA * 2 + i * 32 * BK * 2);
    };
    // the flush below is an FMA with an opaque 1.0 (exact: it rounds t + acc
    // once, like an add) so that each accumulator is updated in place
    float one;
    asm("v_mov_b32 %0, 1.0" : "=v"(one));
    const f32x16_t zero = {};

    // prologue: A stages 0 and 1 into buffers 0 and 1, stage 2 into
    // registers; B stage 0 split, stage 1 in registers
#pragma unroll
    for (int v = 0; v < NSA; ++v) a_load(v, 0, 0 >= nfull);
#pragma unroll
    for (int kc = 0; kc < KPG; ++kc) b_load(kc, 0, 0 >= nfull);
#pragma unroll
    for (int v = 0; v < NSA; ++v) a_store(v, smem);
    if (nk > 1) {
#pragma unroll
      for (int v = 0; v < NSA; ++v) a_load(v, 1, 1 >= nfull);
#pragma unroll
      for (int v = 0; v < NSA; ++v) a_store(v, smem + stage);
    }
#pragma unroll
    for (int kc = 0; kc < KPG; ++kc) b_split(kc);
    if (nk > 1) {
#pragma unroll
      for (int kc = 0; kc < KPG; ++kc) b_load(kc, 1, 1 >= nfull);
    }
    if (nk > 2) {
#pragma unroll
      for (int v = 0; v < NSA; ++v) a_load(v, 2, 2 >= nfull);
    }
    __syncthreads();
    read_a(smem, 0, 0, 0);

    // One stage: TM x KPG block steps (block row outer).  A block's products
    // of the stage form one chain on the matrix cores that starts from zero
    // (smallest products first), and the chain is added to the block's
    // accumulator with one vector add (round to nearest even): the running
    // sums never take a matrix-core accumulation, whose rounding onto a
    // large value drifts.  After the last block, B of the next stage is
    // split into the fragments and refilled from the stage after; A's
    // next-but-one stage is split into LDS and refilled from the stage after
    // that.  The first A fragments of the next stage are read before the
    // barrier.
    constexpr int NSTEP = KPG * TM;
    auto stage = [&](int kt, auto steady) {
      constexpr bool S = decltype(steady)::value;
      const char* cur = smem + (kt % NBUF) * stage_bytes();
      const char* nxt = smem + ((kt + 1) % NBUF) * stage_bytes();
      char* st2 = smem + ((kt + 2) % NBUF) * stage_bytes();
      const bool has1 = S || kt + 1 < nk;
      const bool has2 = S || kt + 2 < nk;
      const bool has3 = S || kt + 3 < nk;
      f32x16_t ch;
#pragma unroll
      for (int s = 0; s < NSTEP; ++s) {
        const int i = s / KPG, kc = s % KPG, sa = s & 1;
        // (the next stage's first step reads set 0; with an odd step count
        // the last step itself uses set 0, which is refilled only once this
        // step's products are issued)
        if (s + 1 < NSTEP)
          read_a(cur, (s + 1) % KPG, (s + 1) / KPG, sa ^ 1);
        else if (NSTEP % 2 == 0 && has1)
          read_a(nxt, 0, 0, 0);
#pragma unroll
        for (int q = 0; q < 6; ++q) {
          const int pa = q == 0 ? 1 : q == 1 ? 0 : q == 2 ? 2 : q == 3 ? 0 : q == 4 ? 1 : 0;
          const int pb = q == 0 ? 1 : q == 1 ? 2 : q == 2 ? 0 : q == 3 ? 1 : q == 4 ? 0 : 0;
          ch = __builtin_amdgcn_mfma_f32_32x32x16_bf16(af[sa][pa], bf[kc][pb], (kc == 0 && q == 0) ? zero : ch, 0,
                                                       0, 0);
        }
        if (s == NSTEP - 1 && NSTEP % 2 == 1 && has1) read_a(nxt, 0, 0, 0);
        if (kc == KPG - 1) {
#pragma unroll
          for (int r = 0; r < 16; ++r) acc[i][r] = __builtin_fmaf(ch[r], one, acc[i][r]);
        }
        if (s == NSTEP - 1) {
          // this stage's last use of B is issued
#pragma unroll
          for (int k2 = 0; k2 < KPG; ++k2) {
            if (has1) b_split(k2);
            if (has2) b_load(k2, kt + 2, !S && kt + 2 >= nfull);
          }
        }
        // A: slot v after step (2 v + 1) (spread over the stage)
#pragma unroll
        for (int v = 0; v < NSA; ++v)
          if (s == (2 * v + 1) % NSTEP) {
            if (has2) a_store(v, st2);
            if (has3) a_load(v, kt + 3, !S && kt + 3 >= nfull);
          }
      }
      __syncthreads();
    };

    using T_ = std::integral_constant<bool, true>;
    using F_ = std::integral_constant<bool, false>;
    int kt = 0;
    for (; kt + 3 < nfull; ++kt) stage(kt, T_());
    for (; kt < nk; ++kt) stage(kt, F_());

    if constexpr (WK > 1) {
      // the second k group's sums are added into the first's through LDS
      // (free after the last stage barrier)
      static_assert(WK == 2, "two k groups");
      float* red = reinterpret_cast<float*>(smem);
      const int wc = wave % NWC;
      if (kg == 1) {
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
          for (int r = 0; r < 16; ++r) red[((wc * TM + i) * 16 + r) * 64 + lane] = acc[i][r];
      }
      __syncthreads();
      if (kg == 0) {
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
          for (int r = 0; r < 16; ++r) acc[i][r] += red[((wc * TM + i) * 16 + r) * 64 + lane];
      }
      __syncthreads();
    }

    int64_t* offm = reinterpret_cast<int64_t*>(smem);
    int64_t* offn = offm + BM;
    for (int e = tid; e < BM + BN; e += NT) {
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
    float* C = d.c + bz * d.c_bs;
    float amax = 0.f;
    const bool mvec = d.c_mode == STORE_MVEC;
    const bool scaled = scale != 1.0f;
    const int nl = wn_off + lr;
    const bool nok = kg == 0 && n0 + nl < d.N;
    const int64_t on = offn[nl];
#pragma unroll
    for (int i = 0; i < TM; ++i) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int ml = 32 * i + 8 * q + 4 * lh;
        f32x4_t v = {acc[i][4 * q + 0], acc[i][4 * q + 1], acc[i][4 * q + 2], acc[i][4 * q + 3]};
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
    if (d.c_absmax) {
#pragma unroll
      for (int o = 32; o >= 1; o >>= 1) amax = fmaxf(amax, __shfl_xor(amax, o, 64));
      if (lane == 0) atomicMax(d.c_absmax + bz, __float_as_uint(amax));
    }
  }
  __device__ static constexpr int stage_bytes() { return stage; }
};

template <int BM, int BN, int BMODE, int WK>
__global__ void __launch_bounds__(BN / 32 * WK * 64) __attribute__((amdgpu_waves_per_eu(2, 2)))
    split_gemm_p_kernel(const GemmDesc d) {
  __shared__ __attribute__((aligned(16))) char smem[SplitGemmP<BM, BN, BMODE, WK>::lds_bytes];
  SplitGemmP<BM, BN, BMODE, WK>::run(d, blockIdx.x, blockIdx.z, smem);
}

// Eight waves, two per SIMD: a wave holds at most 256 registers, 160 of them
// the two accumulators of its 160 x 32 strip.
template <int BM, int BN, int WN, int BMODE>
__global__ void __launch_bounds__(WN * 64) __attribute__((amdgpu_waves_per_eu(2, 2)))
    split_gemm_kernel(const GemmDesc d) {
  __shared__ __attribute__((aligned(16))) char smem[SplitGemm<BM, BN, WN, BMODE>::lds_bytes];
  SplitGemm<BM, BN, WN, BMODE>::run(d, blockIdx.x, blockIdx.z, smem);
}

}  // namespace tn
