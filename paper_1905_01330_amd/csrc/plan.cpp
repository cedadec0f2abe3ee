// Host validation, index-group planning and the pairwise-contraction entry
// points (tn_contract_between, tn_trace_edge, tn_outer_product).
#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <vector>

#include "internal.h"

namespace tn {

static thread_local char g_err[512] = "";

void set_error(const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
}

int32_t fail(int32_t code, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
  return code;
}

int32_t hip_check(hipError_t e, const char* what) {
  if (e == hipSuccess) return TN_OK;
  return fail(TN_ERR_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

// ---------------------------------------------------------------------------
// tensors

int32_t check_tensor(const tn_tensor* t, const char* name, int32_t dtype) {
  if (!t) return fail(TN_ERR_INVALID_ARGUMENT, "%s is NULL", name);
  if (t->rank < 0 || t->rank > TN_MAX_RANK) return fail(TN_ERR_INVALID_ARGUMENT, "%s: rank %d out of range", name, t->rank);
  if (dtype >= 0 && t->dtype != dtype)
    return fail(TN_ERR_UNSUPPORTED, "%s: dtype %d not supported here (want %d)", name, t->dtype, dtype);
  if (t->dtype != TN_F32 && t->dtype != TN_F64 && t->dtype != TN_C64)
    return fail(TN_ERR_UNSUPPORTED, "%s: unknown dtype %d", name, t->dtype);
  if (!t->data) return fail(TN_ERR_INVALID_ARGUMENT, "%s: data is NULL", name);
  for (int i = 0; i < t->rank; ++i) {
    if (t->shape[i] < 1) return fail(TN_ERR_INVALID_ARGUMENT, "%s: shape[%d] = %lld < 1", name, i, (long long)t->shape[i]);
    if (t->stride[i] < 0) return fail(TN_ERR_INVALID_ARGUMENT, "%s: stride[%d] < 0", name, i);
    if (t->shape[i] >= (1ll << 31)) return fail(TN_ERR_UNSUPPORTED, "%s: shape[%d] too large", name, i);
  }
  return TN_OK;
}

int64_t numel(const tn_tensor& t) {
  int64_t n = 1;
  for (int i = 0; i < t.rank; ++i) n *= t.shape[i];
  return n;
}

void byte_extent(const tn_tensor& t, uintptr_t& lo, uintptr_t& hi) {
  int64_t last = 0;
  for (int i = 0; i < t.rank; ++i) last += (t.shape[i] - 1) * t.stride[i];
  const int64_t es = (t.dtype == TN_F64 || t.dtype == TN_C64) ? 8 : 4;
  lo = reinterpret_cast<uintptr_t>(t.data);
  hi = lo + (uintptr_t)((last + 1) * es);
}

bool overlaps(const tn_tensor& a, const tn_tensor& b) {
  uintptr_t alo, ahi, blo, bhi;
  byte_extent(a, alo, ahi);
  byte_extent(b, blo, bhi);
  return alo < bhi && blo < ahi;
}

bool has_internal_overlap(const tn_tensor& t) {
  std::vector<std::pair<int64_t, int64_t>> ax;
  for (int i = 0; i < t.rank; ++i)
    if (t.shape[i] > 1) ax.push_back({t.stride[i], t.shape[i]});
  std::sort(ax.begin(), ax.end());
  int64_t reach = 0;  // largest offset reachable by the inner axes
  for (auto& p : ax) {
    if (p.first <= reach) return true;
    reach += (p.second - 1) * p.first;
  }
  return false;
}

tn_tensor make_view(void* data, int32_t dtype, std::initializer_list<int64_t> shape) {
  tn_tensor t;
  std::memset(&t, 0, sizeof(t));
  t.data = data;
  t.dtype = dtype;
  t.rank = (int32_t)shape.size();
  int i = 0;
  for (int64_t s : shape) t.shape[i++] = s;
  int64_t st = 1;
  for (int k = t.rank - 1; k >= 0; --k) {
    t.stride[k] = st;
    st *= t.shape[k];
  }
  return t;
}

tn_tensor contiguous_view(void* data, int32_t dtype, int32_t rank, const int64_t* shape) {
  tn_tensor t;
  std::memset(&t, 0, sizeof(t));
  t.data = data;
  t.dtype = dtype;
  t.rank = rank;
  int64_t st = 1;
  for (int k = rank - 1; k >= 0; --k) {
    t.shape[k] = shape[k];
    t.stride[k] = st;
    st *= shape[k];
  }
  return t;
}

// ---------------------------------------------------------------------------
// index groups

void set_fast_div(Group& g) {
  for (int i = 0; i < g.n; ++i) {
    uint32_t d = g.dim[i];
    uint32_t shr = 0;
    while (shr < 32 && (1ull << shr) < d) ++shr;
    uint64_t mul = ((1ull << 32) * ((1ull << shr) - d)) / d + 1;
    g.mul[i] = (uint32_t)mul;
    g.shr[i] = shr;
  }
}

void build_group(std::vector<AxisSpec> axes, int primary, int n_strides, Group& g) {
  std::memset(&g, 0, sizeof(g));
  std::vector<AxisSpec> a;
  for (auto& x : axes)
    if (x.dim > 1) a.push_back(x);
  // outer axes first: descending stride in the primary tensor, then the others
  std::stable_sort(a.begin(), a.end(), [&](const AxisSpec& p, const AxisSpec& q) {
    if (p.s[primary] != q.s[primary]) return p.s[primary] > q.s[primary];
    for (int t = 0; t < n_strides; ++t)
      if (p.s[t] != q.s[t]) return p.s[t] > q.s[t];
    return false;
  });
  std::vector<AxisSpec> m;
  for (auto& x : a) {
    if (!m.empty()) {
      AxisSpec& o = m.back();
      bool ok = true;
      for (int t = 0; t < n_strides; ++t)
        if (o.s[t] != x.s[t] * x.dim) ok = false;
      if (ok && o.dim * x.dim < (1ll << 31)) {
        o.dim *= x.dim;
        for (int t = 0; t < n_strides; ++t) o.s[t] = x.s[t];
        continue;
      }
    }
    m.push_back(x);
  }
  g.n = (int32_t)m.size();
  for (int i = 0; i < g.n; ++i) {
    g.dim[i] = (uint32_t)m[i].dim;
    for (int t = 0; t < 3; ++t) g.s[t][i] = t < n_strides ? m[i].s[t] : 0;
  }
  set_fast_div(g);
}

static int64_t group_size(const Group& g) {
  int64_t n = 1;
  for (int i = 0; i < g.n; ++i) n *= g.dim[i];
  return n;
}

// can operand `t` (stride index `ti`) be read as aligned float4 runs along group `inner`
// 16-byte gathers along the unit-stride axis of `inner`.  The loads need
// only 4-byte alignment (gfx950 runs global vector loads unaligned), so only
// the run structure matters: every micro-block of four stays inside one run
// of the innermost axis, or, for an index with a single axis (tail_ok), a
// partial last micro-block is read element by element.
static bool vec4_load_ok(const Group& inner, int ti, bool tail_ok) {
  if (inner.n < 1) return false;
  const int last = inner.n - 1;
  if (inner.s[ti][last] != 1) return false;
  return inner.dim[last] % 4 == 0 || (tail_ok && inner.n == 1);
}

// 16-byte stores of four consecutive rows of C: aligned runs of four
static bool vec4_ok(const Group& inner, int ti, const Group& other, int oi, const void* ptr, int64_t bstride) {
  if (inner.n < 1) return false;
  const int last = inner.n - 1;
  if (inner.s[ti][last] != 1 || inner.dim[last] % 4 != 0) return false;
  for (int i = 0; i < last; ++i)
    if (inner.s[ti][i] % 4) return false;
  for (int i = 0; i < other.n; ++i)
    if (other.s[oi][i] % 4) return false;
  if (reinterpret_cast<uintptr_t>(ptr) % 16) return false;
  if (bstride % 4) return false;
  return true;
}

// innermost row index unit-stride: the gather reads along rows
static bool mn_scalar_ok(const Group& rows, int ti) {
  return rows.n >= 1 && rows.s[ti][rows.n - 1] == 1;
}

void choose_modes(GemmDesc& d) {
  d.a_mode = vec4_load_ok(d.gk, 0, true) ? LOAD_KVEC
           : vec4_load_ok(d.gm, 0, true) ? LOAD_MNVEC
           : mn_scalar_ok(d.gm, 0)                   ? LOAD_MNSCALAR
                                                     : LOAD_GENERIC;
  d.b_mode = vec4_load_ok(d.gk, 1, true) ? LOAD_KVEC
           : vec4_load_ok(d.gn, 0, true) ? LOAD_MNVEC
           : mn_scalar_ok(d.gn, 0)                   ? LOAD_MNSCALAR
                                                     : LOAD_GENERIC;
  d.c_mode = vec4_ok(d.gm, 1, d.gn, 1, d.c, d.c_bs) ? STORE_MVEC : STORE_SCALAR;
}

int32_t plan_gemm(const tn_tensor& a, const tn_tensor& b, int32_t n_pairs, const int32_t* axes_a,
                  const int32_t* axes_b, const tn_tensor& out, GemmDesc& d) {
  std::memset(&d, 0, sizeof(d));
  bool ca[TN_MAX_RANK] = {false}, cb[TN_MAX_RANK] = {false};
  std::vector<AxisSpec> km, kn, kk;
  for (int p = 0; p < n_pairs; ++p) {
    ca[axes_a[p]] = true;
    cb[axes_b[p]] = true;
    kk.push_back({a.shape[axes_a[p]], {a.stride[axes_a[p]], b.stride[axes_b[p]], 0}});
  }
  int o = 0;
  for (int i = 0; i < a.rank; ++i)
    if (!ca[i]) {
      km.push_back({a.shape[i], {a.stride[i], out.stride[o], 0}});
      ++o;
    }
  for (int j = 0; j < b.rank; ++j)
    if (!cb[j]) {
      kn.push_back({b.shape[j], {b.stride[j], out.stride[o], 0}});
      ++o;
    }
  build_group(km, 0, 2, d.gm);
  build_group(kn, 0, 2, d.gn);
  // K order: innermost = the axis contiguous in A if there is one, else in B
  bool a_unit = false, b_unit = false;
  for (auto& x : kk) {
    if (x.s[0] == 1 && x.dim > 1) a_unit = true;
    if (x.s[1] == 1 && x.dim > 1) b_unit = true;
  }
  build_group(kk, (!a_unit && b_unit) ? 1 : 0, 2, d.gk);
  const int64_t M = group_size(d.gm), N = group_size(d.gn), K = group_size(d.gk);
  if (M >= (1ll << 31) || N >= (1ll << 31) || K >= (1ll << 31))
    return fail(TN_ERR_UNSUPPORTED, "contraction index larger than 2^31");
  d.a = static_cast<const float*>(a.data);
  d.b = static_cast<const float*>(b.data);
  d.c = static_cast<float*>(out.data);
  d.M = (int32_t)M;
  d.N = (int32_t)N;
  d.K = (int32_t)K;
  d.batch = 1;
  choose_modes(d);
  return TN_OK;
}

// ---------------------------------------------------------------------------
// entry points

static int32_t check_prec(int32_t prec) {
  if (prec < TN_PREC_FP32 || prec > TN_PREC_SPLIT_BF16_3P) return fail(TN_ERR_UNSUPPORTED, "unknown precision %d", prec);
  return TN_OK;
}

int32_t contract_between_impl(const tn_tensor* a, const tn_tensor* b, int32_t n_pairs, const int32_t* axes_a,
                              const int32_t* axes_b, tn_tensor* out, void* scratch, size_t scratch_bytes,
                              int32_t prec, hipStream_t st) {
  TN_TRY(check_tensor(a, "a", TN_F32));
  TN_TRY(check_tensor(b, "b", TN_F32));
  TN_TRY(check_tensor(out, "out", TN_F32));
  TN_TRY(check_prec(prec));
  if (n_pairs < 0 || n_pairs > a->rank || n_pairs > b->rank)
    return fail(TN_ERR_INVALID_ARGUMENT, "n_pairs = %d out of range", n_pairs);
  if (n_pairs > 0 && (!axes_a || !axes_b)) return fail(TN_ERR_INVALID_ARGUMENT, "axes are NULL");
  bool ua[TN_MAX_RANK] = {false}, ub[TN_MAX_RANK] = {false};
  for (int p = 0; p < n_pairs; ++p) {
    int i = axes_a[p], j = axes_b[p];
    if (i < 0 || i >= a->rank || j < 0 || j >= b->rank) return fail(TN_ERR_INVALID_ARGUMENT, "pair %d: axis out of range", p);
    if (ua[i] || ub[j]) return fail(TN_ERR_INVALID_ARGUMENT, "pair %d: axis repeated", p);
    ua[i] = ub[j] = true;
    if (a->shape[i] != b->shape[j])
      return fail(TN_ERR_SHAPE_MISMATCH, "pair %d: connected dimensions differ (%lld vs %lld)", p,
                  (long long)a->shape[i], (long long)b->shape[j]);
  }
  const int orank = a->rank + b->rank - 2 * n_pairs;
  if (out->rank != orank) return fail(TN_ERR_SHAPE_MISMATCH, "out rank %d, expected %d", out->rank, orank);
  int o = 0;
  for (int i = 0; i < a->rank; ++i)
    if (!ua[i] && out->shape[o++] != a->shape[i]) return fail(TN_ERR_SHAPE_MISMATCH, "out axis %d has the wrong extent", o - 1);
  for (int j = 0; j < b->rank; ++j)
    if (!ub[j] && out->shape[o++] != b->shape[j]) return fail(TN_ERR_SHAPE_MISMATCH, "out axis %d has the wrong extent", o - 1);
  if (overlaps(*out, *a) || overlaps(*out, *b)) return fail(TN_ERR_ALIASING, "out overlaps an input");
  if (has_internal_overlap(*out)) return fail(TN_ERR_INVALID_ARGUMENT, "out view maps two indices to one address");

  GemmDesc d;
  TN_TRY(plan_gemm(*a, *b, n_pairs, axes_a, axes_b, *out, d));
  const bool small_out = d.M == 1 || d.N == 1 || ((int64_t)d.M * d.N <= 256 && d.K >= 4096);
  if (d.K == 1 || small_out) {
    // rank-0/1 results, outer products: wavefront reductions / elementwise products
    ReduceDesc r;
    std::memset(&r, 0, sizeof(r));
    std::vector<AxisSpec> ra, ka;
    for (int i = 0; i < d.gm.n; ++i) ra.push_back({d.gm.dim[i], {d.gm.s[0][i], 0, d.gm.s[1][i]}});
    for (int i = 0; i < d.gn.n; ++i) ra.push_back({d.gn.dim[i], {0, d.gn.s[0][i], d.gn.s[1][i]}});
    for (int i = 0; i < d.gk.n; ++i) ka.push_back({d.gk.dim[i], {d.gk.s[0][i], d.gk.s[1][i], 0}});
    return reduce_from_axes(d.a, d.b, d.c, ra, ka, prec == TN_PREC_BF16, scratch, scratch_bytes, st);
  }
  return launch_gemm(d, prec, st);
}

int32_t reduce_from_axes(const float* x, const float* y, float* out, const std::vector<AxisSpec>& r_axes,
                         const std::vector<AxisSpec>& k_axes, bool bf16_round, void* scratch, size_t scratch_bytes,
                         hipStream_t st) {
  ReduceDesc r;
  std::memset(&r, 0, sizeof(r));
  r.x = x;
  r.y = y;
  r.out = out;
  // outputs ordered by the output tensor's strides so consecutive threads store consecutively
  build_group(r_axes, 2, 3, r.gr);
  build_group(k_axes, 0, 2, r.gk);
  r.R = group_size(r.gr);
  r.K = group_size(r.gk);
  r.bf16_round = bf16_round ? 1 : 0;
  return launch_reduce(r, scratch, scratch_bytes, st);
}

}  // namespace tn

using namespace tn;

extern "C" {

const char* tn_status_string(int32_t s) {
  switch (s) {
    case TN_OK: return "ok";
    case TN_ERR_INVALID_ARGUMENT: return "invalid argument";
    case TN_ERR_SHAPE_MISMATCH: return "shape mismatch";
    case TN_ERR_UNSUPPORTED: return "unsupported";
    case TN_ERR_WORKSPACE_TOO_SMALL: return "workspace too small";
    case TN_ERR_ALIASING: return "output aliases an input";
    case TN_ERR_DEVICE: return "device error";
    default: return "unknown status";
  }
}

const char* tn_last_error(void) { return g_err; }

const char* tn_version(void) { return "tn-mi355x 0.1 gfx950"; }

int32_t tn_contract_between(const tn_tensor* a, const tn_tensor* b, int32_t n_pairs, const int32_t* axes_a,
                            const int32_t* axes_b, tn_tensor* out, void* workspace, size_t ws_bytes, int32_t prec,
                            void* stream) {
  g_err[0] = 0;
  if (ws_bytes > 0 && !workspace) return fail(TN_ERR_INVALID_ARGUMENT, "workspace is NULL but ws_bytes = %zu", ws_bytes);
  return contract_between_impl(a, b, n_pairs, axes_a, axes_b, out, workspace, workspace ? ws_bytes : 0, prec,
                               static_cast<hipStream_t>(stream));
}

int32_t tn_trace_edge(const tn_tensor* a, int32_t axis1, int32_t axis2, tn_tensor* out, void* stream) {
  g_err[0] = 0;
  TN_TRY(check_tensor(a, "a", TN_F32));
  TN_TRY(check_tensor(out, "out", TN_F32));
  if (axis1 < 0 || axis1 >= a->rank || axis2 < 0 || axis2 >= a->rank || axis1 == axis2)
    return fail(TN_ERR_INVALID_ARGUMENT, "trace axes (%d, %d) invalid for rank %d", axis1, axis2, a->rank);
  if (a->shape[axis1] != a->shape[axis2]) return fail(TN_ERR_SHAPE_MISMATCH, "trace axes have different extents");
  if (out->rank != a->rank - 2) return fail(TN_ERR_SHAPE_MISMATCH, "out rank %d, expected %d", out->rank, a->rank - 2);
  std::vector<AxisSpec> ra, ka;
  int o = 0;
  for (int i = 0; i < a->rank; ++i) {
    if (i == axis1 || i == axis2) continue;
    if (out->shape[o] != a->shape[i]) return fail(TN_ERR_SHAPE_MISMATCH, "out axis %d has the wrong extent", o);
    ra.push_back({a->shape[i], {a->stride[i], 0, out->stride[o]}});
    ++o;
  }
  if (overlaps(*out, *a)) return fail(TN_ERR_ALIASING, "out overlaps the input");
  if (has_internal_overlap(*out)) return fail(TN_ERR_INVALID_ARGUMENT, "out view maps two indices to one address");
  ka.push_back({a->shape[axis1], {a->stride[axis1] + a->stride[axis2], 0, 0}});
  return reduce_from_axes(static_cast<const float*>(a->data), nullptr, static_cast<float*>(out->data), ra, ka, false,
                          nullptr, 0, static_cast<hipStream_t>(stream));
}

int32_t tn_outer_product(const tn_tensor* a, const tn_tensor* b, tn_tensor* out, void* stream) {
  g_err[0] = 0;
  return contract_between_impl(a, b, 0, nullptr, nullptr, out, nullptr, 0, TN_PREC_FP32,
                               static_cast<hipStream_t>(stream));
}

}  // extern "C"
