// Host-side internal interfaces of the library.
#pragma once

#include <vector>

#include "common.h"

namespace tn {

// ---- tensors -------------------------------------------------------------
int32_t check_tensor(const tn_tensor* t, const char* name, int32_t dtype);
int64_t numel(const tn_tensor& t);
// [lo, hi) byte range touched by a view (hi = lo for an empty view)
void byte_extent(const tn_tensor& t, uintptr_t& lo, uintptr_t& hi);
bool overlaps(const tn_tensor& a, const tn_tensor& b);
bool has_internal_overlap(const tn_tensor& t);
tn_tensor make_view(void* data, int32_t dtype, std::initializer_list<int64_t> shape);
tn_tensor contiguous_view(void* data, int32_t dtype, int32_t rank, const int64_t* shape);

// ---- GEMM plan (contraction of strided views) ------------------------------
// Builds the GEMM view of a tensordot: M = free axes of a (ascending),
// N = free axes of b (ascending), K = pairs in the given order.  Axes of
// extent 1 are dropped and axes contiguous in every tensor of their group
// are merged; each group is ordered so its most contiguous axis is inner.
int32_t plan_gemm(const tn_tensor& a, const tn_tensor& b, int32_t n_pairs, const int32_t* axes_a,
                  const int32_t* axes_b, const tn_tensor& out, GemmDesc& d);
// (re)select the operand load and store modes after a descriptor's pointers
// or batch strides change
void choose_modes(GemmDesc& d);

// reductions: out[r] = sum_k x * y (y may be null)
struct AxisSpec {
  int64_t dim;
  int64_t s[3];
};
void build_group(std::vector<AxisSpec> axes, int primary, int n_strides, Group& g);
// scratch: nullable device buffer of scratch_bytes (TN_REDUCE_WORKSPACE_BYTES
// enables the split reduction of few long sums)
constexpr size_t kReduceScratchBytes = TN_REDUCE_WORKSPACE_BYTES;
int32_t launch_reduce(ReduceDesc& d, void* scratch, size_t scratch_bytes, hipStream_t st);
int32_t reduce_from_axes(const float* x, const float* y, float* out, const std::vector<AxisSpec>& r_axes,
                         const std::vector<AxisSpec>& k_axes, bool bf16_round, void* scratch, size_t scratch_bytes,
                         hipStream_t st);

// ---- GEMM launch -----------------------------------------------------------
int32_t launch_gemm(GemmDesc& d, int32_t prec, hipStream_t st);
// While one of these lives on a thread, launch_gemm on that thread never
// times tile candidates (the cached or heuristic tile is used): timing
// creates HIP events, which the allocation-free entry points avoid.
struct NoTimingScope {
  NoTimingScope();
  ~NoTimingScope();
  bool prev;
};
// While one of these lives on a thread, launch_gemm on that thread serves
// GEMMs that share the chip with a concurrent stream (the two halves of a
// two-directional sweep or inner product): tiles are estimated for half the
// compute units, timed as two copies running at once, and cached apart
// from the same GEMM issued alone.
struct SharedChipScope {
  explicit SharedChipScope(bool on = true);
  ~SharedChipScope();
  bool prev;
};
// While one of these lives on a thread, launch_gemm on that thread may cut
// a GEMM that fills few compute units into k-slices: the slices run as one
// batched launch into dense partial results in `scratch` (device, at least
// `floats` floats; the caller's, not shared with concurrent work) and a
// second kernel adds them in slice order into C.  The tuner times the slice
// counts beside the tiles; the choice is cached with the tile (the cache
// value is tile + 100 log2(slices)).
struct SplitKScope {
  // at most 2^max_lg slices a GEMM (capped at 64)
  SplitKScope(float* scratch, size_t floats, int max_lg = 2);
  ~SplitKScope();
  float* prev_p;
  size_t prev_n;
  int prev_lg;
};
// Householder QR of a column-major m x n FP64 matrix (m >= n, m <= 2048 when
// householder_qr_fits): factorised in place, with the panels' triangular
// factors in tf (householder_tf_doubles(n) doubles) and tau (n doubles);
// householder_apply_q replaces y (m x ncols, column-major) by Q y.
bool householder_qr_fits(int64_t m);
size_t householder_tf_doubles(int64_t n);
int32_t householder_qr(double* xc, int m, int n, double* tau, double* tf, hipStream_t st);
int32_t householder_apply_q(const double* xc, int m, int n, const double* tf, double* y, int ncols, hipStream_t st);
// K <= 32 with N or M <= 16 (and no batch, scale or max-abs): the HBM-bound path
bool gemm_small_fits(const GemmDesc& d);
int32_t launch_gemm_small(const GemmDesc& d, int32_t prec, hipStream_t st);
int32_t launch_gemm_cfg(GemmDesc& d, int32_t prec, int cfg, hipStream_t st);
int gemm_num_cfgs();

// grouped GEMM over compact 2-D problems (uneven batches)
struct Gemm2D {
  const float* a;
  const float* b;
  float* c;
  int32_t M, N, K;
  int64_t sam, sak, sbk, sbn, scm, scn;
  const uint32_t* a_scale_bits;
  uint32_t* c_absmax;
};
// variant: 0 run-time gathers; 1..4 fast gathers, for launches whose every
// problem passes grouped_variant with that value
int grouped_variant(const Gemm2D& p);
int32_t launch_gemm_grouped(const Gemm2D* dev_probs, const int32_t* dev_tile_start, int32_t n_probs,
                            int32_t total_tiles, int32_t prec, int cfg, int variant, hipStream_t st);
int grouped_tile_m(int cfg);
// the library's side stream for the caller's stream s on the current device
// (s in, side stream out): one of a pool of four per device (created on first
// use, default priority, never destroyed), assigned to caller streams in
// turn and kept, so calls on up to four different streams do not queue
// behind each other's side work.  Work is forked from and joined back into
// the caller's stream by events.
int32_t side_stream(hipStream_t& s);
// grouped tile configuration pinned by tn_tune_force_grouped_config, or -1
int forced_grouped_cfg();
// the tuning level when timing is allowed on st now (not disabled on this
// thread, stream not capturing), else 0
int tune_timing_level(hipStream_t st);
// tuned grouped tile of a step (signature, precision), or -1; record a choice
// (timed choices are appended to the tile cache file)
int grouped_tune_get(uint64_t sig, int prec);
void grouped_tune_put(uint64_t sig, int prec, int cfg, bool timed);
int grouped_tile_n(int cfg);

// ---- complex contraction on the real path (complex.hip) -----------------------
size_t c64_workspace_bytes(const tn_tensor& b);
int32_t contract_c64_impl(const tn_tensor* a, const tn_tensor* b, int32_t n_pairs, const int32_t* axes_a,
                          const int32_t* axes_b, int conj_a, int conj_b, tn_tensor* out, void* workspace,
                          size_t ws_bytes, int32_t prec, hipStream_t st);

// ---- contraction entry used by the network driver -----------------------------
int32_t contract_between_impl(const tn_tensor* a, const tn_tensor* b, int32_t n_pairs, const int32_t* axes_a,
                              const int32_t* axes_b, tn_tensor* out, void* scratch, size_t scratch_bytes,
                              int32_t prec, hipStream_t st);

}  // namespace tn
