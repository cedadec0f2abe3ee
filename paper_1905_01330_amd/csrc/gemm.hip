// Contraction GEMM: kernel instantiations, tile selection, autotuner and the
// grouped launch used for uneven batches of small problems.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "gemm_inst.h"

namespace tn {

// ---------------------------------------------------------------------------
// tile configurations

struct Cfg {
  int bm, bn, bk, wm, wn;
  float eff;          // relative per-tile efficiency used by the heuristic
  int wk = 1;         // k-slice groups of wm x wn waves
  int split = 0;      // lean-stage split-BF16 kernel kind (gemm_split.hip), 0: general kernel
  int fallback = -1;  // general configuration of the same tile shape, for problems the kind cannot take
  bool swap = false;  // run on the transposed problem C^T = B^T A^T (operands exchanged)
};

// eff: relative per-tile throughput measured on the bulk environment-sweep
// shapes (chi = 1024); the heuristic divides the padded tile work by it
static const Cfg kCfgs[] = {
    {256, 128, 16, 2, 2, 0.75f}, {128, 256, 16, 2, 2, 0.80f}, {128, 128, 16, 2, 2, 1.00f},
    {128, 128, 32, 2, 2, 0.95f}, {128, 64, 32, 2, 2, 0.70f},  {64, 128, 32, 2, 2, 0.70f},
    {64, 64, 32, 2, 2, 0.55f},   {32, 32, 32, 1, 1, 0.25f},  {160, 128, 16, 1, 4, 1.00f},
    {128, 160, 16, 4, 1, 1.00f},   {160, 256, 32, 1, 8, 2.00f}, {256, 160, 32, 8, 1, 2.00f},
    {128, 160, 32, 4, 1, 1.60f, 2}, {160, 128, 32, 1, 4, 1.60f, 2}, {64, 64, 64, 2, 2, 0.45f, 2},
    {64, 64, 64, 2, 2, 0.55f},
    // lean-stage split-BF16 kernels (split-BF16 precision, k-contiguous A,
    // B along k or n, K % 8 == 0, 31-bit byte offsets); tiles as 10 and 13
    {160, 256, 32, 1, 8, 2.30f, 1, 1, 10}, {160, 256, 32, 1, 8, 2.20f, 1, 2, 10},
    {160, 128, 32, 1, 4, 1.75f, 2, 3, 13},
    // the same on the exchanged operands (B k-contiguous); tiles as 11 and 12
    {256, 160, 32, 8, 1, 2.30f, 1, 1, 11, true}, {256, 160, 32, 8, 1, 2.20f, 1, 2, 11, true},
    {128, 160, 32, 4, 1, 1.75f, 2, 3, 12, true},
};
static constexpr int kNumCfgs = sizeof(kCfgs) / sizeof(kCfgs[0]);

int gemm_num_cfgs() { return kNumCfgs; }

// fast gathers need one merged K axis and vector-friendly layouts on both operands
static int gemm_variant(const GemmDesc& d) {
  if (d.gk.n != 1 || d.a_mode == LOAD_GENERIC || d.b_mode == LOAD_GENERIC || d.a_mode == LOAD_MNSCALAR ||
      d.b_mode == LOAD_MNSCALAR)
    return 0;
  // the fast m/n-contiguous gathers read blocks of four rows; a partial last
  // block (one row axis, M % 4 != 0) needs M >= 4 and a k stride >= 4,
  // since the stages before the last may read up to three elements past it
  auto fits = [](const Group& g, int64_t sk) {
    return g.dim[g.n - 1] % 4 == 0 || (g.n == 1 && g.dim[0] >= 4 && sk >= 4);
  };
  if ((d.a_mode == LOAD_MNVEC && !fits(d.gm, d.gk.s[0][0])) || (d.b_mode == LOAD_MNVEC && !fits(d.gn, d.gk.s[1][0])))
    return 0;
  return 1 + (d.a_mode == LOAD_MNVEC ? 2 : 0) + (d.b_mode == LOAD_MNVEC ? 1 : 0);
}

// the lean-stage split-BF16 kernels take the split precision with one
// merged contracted axis, A read along it in 16-byte loads, K a multiple of 8
// (whole 8-k runs) and every element of one batch entry within a 31-bit byte
// offset of the view's base (buffer loads).  B is read in 16-byte loads when
// it is k-contiguous, else one element per lane along k (lanes along n).
static bool split_ok(const GemmDesc& d, int prec) {
  if (prec != TN_PREC_SPLIT_BF16 || d.gk.n != 1 || d.a_mode != LOAD_KVEC || d.K % 8 != 0) return false;
  // their 16-byte buffer loads (A, and B when read along k) take 16-byte
  // aligned rows
  auto aligned = [](const void* p, const Group& rows, int64_t bs) {
    if (reinterpret_cast<uintptr_t>(p) % 16 || bs % 4) return false;
    for (int i = 0; i < rows.n; ++i)
      if (rows.s[0][i] % 4) return false;
    return true;
  };
  if (!aligned(d.a, d.gm, d.a_bs)) return false;
  if (d.b_mode == LOAD_KVEC && !aligned(d.b, d.gn, d.b_bs)) return false;
  auto extent = [](const Group& g, int t) {
    int64_t e = 0;
    for (int i = 0; i < g.n; ++i) e += (int64_t)(g.dim[i] - 1) * g.s[t][i];
    return e;
  };
  const int64_t ea = extent(d.gm, 0) + extent(d.gk, 0) + 8;
  const int64_t eb = extent(d.gn, 0) + extent(d.gk, 1) + 8;
  return ea * 4 < (1ll << 31) && eb * 4 < (1ll << 31);
}

// C^T = B^T A^T: the operands and the M and N groups exchanged (the output
// strides travel with their groups), modes re-derived
static GemmDesc exchanged(const GemmDesc& d) {
  GemmDesc e = d;
  e.a = d.b;
  e.b = d.a;
  e.M = d.N;
  e.N = d.M;
  e.a_bs = d.b_bs;
  e.b_bs = d.a_bs;
  e.gm = d.gn;
  e.gn = d.gm;
  for (int i = 0; i < kMaxAxes; ++i) {
    e.gk.s[0][i] = d.gk.s[1][i];
    e.gk.s[1][i] = d.gk.s[0][i];
  }
  choose_modes(e);
  return e;
}

// lean: run the lean kind of cfg (the caller has checked that it applies to d)
static GemmFn pick_fn(const GemmDesc& d, int prec, int cfg, bool lean) {
  const Cfg& g = kCfgs[cfg];
  if (g.split) {
    if (lean) return split_fn(g.split, d.b_mode == LOAD_KVEC ? LOAD_KVEC : LOAD_MNVEC);
    cfg = g.fallback;
  }
  return gemm_fn_prec(prec, cfg, gemm_variant(d));
}

// grouped configurations: 0 -> 128x128, 1 -> 64x64, 2 -> 32x32, 3 -> 64x64 in two k-slices
static const int kGroupedCfg[5] = {3, 15, 7, 14, 10};
int grouped_tile_m(int cfg) { return kCfgs[kGroupedCfg[cfg]].bm; }
int grouped_tile_n(int cfg) { return kCfgs[kGroupedCfg[cfg]].bn; }

static GroupedFn pick_grouped(int prec, int cfg, int variant) { return grouped_fn_prec(prec, cfg, variant); }

static std::atomic<int> g_forced_cfg{-1};
static std::atomic<int> g_forced_grouped{-1};

int forced_grouped_cfg() { return g_forced_grouped.load(); }

// eight-wave tiles larger than 64 x 64 have a fixed 256-register budget that
// the run-time-mode gathers exceed: they serve the fast gathers only
// (the lean-stage kinds only where they apply)
static bool cfg_allowed(const GemmDesc& d, int prec, int c) {
  const Cfg& g = kCfgs[c];
  if (g.split) return split_ok(g.swap ? exchanged(d) : d, prec);
  return g.wm * g.wn * g.wk < 8 || g.bm * g.bn <= 64 * 64 || gemm_variant(d) != 0;
}

// set while the calling thread issues GEMMs that share the chip with a
// concurrent stream (the two directions of a sweep, the two ends of an
// inner product)
static thread_local bool g_shared = false;

SharedChipScope::SharedChipScope(bool on) : prev(g_shared) { g_shared = prev || on; }
SharedChipScope::~SharedChipScope() { g_shared = prev; }

// k-slice scratch of the calling thread (SplitKScope), in floats
static thread_local float* g_splitk = nullptr;
static thread_local size_t g_splitk_floats = 0;
static thread_local int g_splitk_maxlg = 0;

// A choice is a tile configuration and a k-slice count 2^lg, kept as
// cfg + 100 lg (lg = 0: the GEMM runs whole).
static int choice_cfg(int v) { return v % 100; }
static int choice_lg(int v) { return v / 100; }
constexpr int kMaxSliceLg = 6;

SplitKScope::SplitKScope(float* scratch, size_t floats, int max_lg)
    : prev_p(g_splitk), prev_n(g_splitk_floats), prev_lg(g_splitk_maxlg) {
  g_splitk = scratch;
  g_splitk_floats = floats;
  g_splitk_maxlg = std::max(0, std::min(max_lg, kMaxSliceLg));
}
SplitKScope::~SplitKScope() {
  g_splitk = prev_p;
  g_splitk_floats = prev_n;
  g_splitk_maxlg = prev_lg;
}

// the most k-slices (log 2) the calling thread's scope allows
static int max_slice_lg() { return g_splitk ? g_splitk_maxlg : 0; }

// Whether the GEMM can run as 2^lg k-slices into the scratch: the slices
// cut the outermost contracted axis evenly (a slice is then a pointer
// offset; with several contracted axes, one that keeps 16-byte alignment),
// no batch (the scale and |C| maximum, if any, are the single entry's and
// move to the sum kernel), slices of whole 16-k steps and at least 64 long,
// and room for the 2^lg dense M x N partial results.
static bool slices_ok(const GemmDesc& d, int lg) {
  if (lg == 0) return true;
  const int S = 1 << lg;
  if (!g_splitk || lg > max_slice_lg() || d.batch != 1 || d.gk.n < 1 || d.gk.dim[0] % S != 0) return false;
  const int64_t d0 = d.gk.dim[0] / S;
  if (d.gk.n > 1 && ((d0 * d.gk.s[0][0]) % 4 != 0 || (d0 * d.gk.s[1][0]) % 4 != 0)) return false;
  return d.K % (16 * S) == 0 && d.K / S >= 64 && (size_t)S * (size_t)d.M * (size_t)d.N <= g_splitk_floats;
}

// The slices as a batch of S GEMMs: slice z contracts k in [z K/S, (z+1) K/S)
// (A and B advanced by dim0/S steps of the outermost contracted axis, dim0
// its extent) into the dense M x N partial z of the scratch.
static GemmDesc slice_desc(const GemmDesc& d, int S) {
  GemmDesc x = d;
  const uint32_t d0 = d.gk.dim[0] / (uint32_t)S;
  x.K = d.K / S;
  x.gk.dim[0] = d0;
  set_fast_div(x.gk);
  x.batch = S;
  x.a_bs = (int64_t)d0 * d.gk.s[0][0];
  x.b_bs = (int64_t)d0 * d.gk.s[1][0];
  x.c = g_splitk;
  x.c_bs = (int64_t)d.M * d.N;
  x.a_scale_bits = nullptr;   // applied to the sum (an exact power of two)
  x.c_absmax = nullptr;       // taken over the sum
  int64_t st = d.N;
  for (int i = x.gm.n - 1; i >= 0; --i) {
    x.gm.s[1][i] = st;
    st *= x.gm.dim[i];
  }
  st = 1;
  for (int i = x.gn.n - 1; i >= 0; --i) {
    x.gn.s[1][i] = st;
    st *= x.gn.dim[i];
  }
  choose_modes(x);
  return x;
}

// C[m, n] = the partials' sum over the slices in slice order (deterministic),
// times the GEMM's 2^-e scale if it has one, stored through C's index groups;
// the GEMM's |C| maximum (if any) is taken over these values
__global__ void __launch_bounds__(256) slice_sum_kernel(const float* __restrict__ part, int S, int M, int N,
                                                        float* __restrict__ c, const Group gm, const Group gn,
                                                        const uint32_t* __restrict__ scale_bits,
                                                        uint32_t* __restrict__ absmax) {
  const int64_t MN = (int64_t)M * N;
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  float a = 0.f;
  if (i < MN) {
    const int m = (int)(i / N), n = (int)(i - (int64_t)m * N);
    float s = part[i];
    for (int z = 1; z < S; ++z) s += part[z * MN + i];
    if (scale_bits) s *= pow2_inverse_scale(scale_bits[0]);
    int64_t om[1], on[1];
    group_offsets<1>(gm, (uint32_t)m, om, 1);
    group_offsets<1>(gn, (uint32_t)n, on, 1);
    c[om[0] + on[0]] = s;
    a = fabsf(s);
  }
  if (absmax) {   // uniform over the grid: every lane reaches the shuffles
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) a = fmaxf(a, __shfl_xor(a, o, 64));
    if ((threadIdx.x & 63) == 0) atomicMax(absmax, __float_as_uint(a));
  }
}

static int heuristic_cfg(const GemmDesc& d, int prec) {
  const int forced = g_forced_cfg.load();
  if (forced >= 0) return forced;
  // one workgroup per compute unit for the large tiles; a GEMM that shares
  // the chip with a concurrent stream counts on half of them
  const int kSlots = g_shared ? 128 : 256;
  double best = 1e300;
  int best_c = 7;   // 32 x 32 tiles fit every problem
  for (int c = 0; c < kNumCfgs; ++c) {
    if (!cfg_allowed(d, prec, c)) continue;
    const Cfg& g = kCfgs[c];
    const int64_t tiles = (int64_t)((d.M + g.bm - 1) / g.bm) * ((d.N + g.bn - 1) / g.bn) * d.batch;  // bm x bn as the caller's M x N
    const int64_t rounds = (tiles + kSlots - 1) / kSlots;
    // rounds of full-chip occupancy times the work of one tile over its efficiency
    const double est = (double)rounds * g.bm * g.bn / g.eff;
    if (est < best * 0.999) {
      best = est;
      best_c = c;
    }
  }
  return best_c;
}

// ---------------------------------------------------------------------------
// autotune cache

using TuneKey = std::tuple<int, int, int, int, int, int, int, int, int>;
static std::mutex g_tune_mu;
static int g_tune_level = 0;
static std::map<TuneKey, int> g_tune_cache;
// grouped launches of the uneven batch: (step signature, precision) -> grouped tile
static std::map<std::pair<uint64_t, int>, int> g_grouped_cache;
static std::string g_tune_path;   // persisted cache file ("" = memory only)
static thread_local int g_last_choice = -1;
static thread_local bool g_no_timing = false;

NoTimingScope::NoTimingScope() : prev(g_no_timing) { g_no_timing = true; }
NoTimingScope::~NoTimingScope() { g_no_timing = prev; }
static std::once_flag g_env_once;
static bool g_log = false;

// "M N K batch amode bmode cmode prec groups -> cfg" per line, and
// "G signature prec -> cfg" (signature in hex) for the grouped launches;
// caller holds g_tune_mu
static void load_cache_file_locked() {
  if (g_tune_path.empty()) return;
  FILE* f = std::fopen(g_tune_path.c_str(), "r");
  if (!f) return;
  char line[256];
  while (std::fgets(line, sizeof(line), f)) {
    if (line[0] == 'G') {
      unsigned long long sig = 0;
      int pr = 0, c = -1;
      if (std::sscanf(line, "G %llx %d -> %d", &sig, &pr, &c) == 3 && c >= 0 && c < 5)
        g_grouped_cache[std::make_pair((uint64_t)sig, pr)] = c;
      continue;
    }
    int v[10];
    if (std::sscanf(line, "%d %d %d %d %d %d %d %d %d -> %d", &v[0], &v[1], &v[2], &v[3], &v[4], &v[5], &v[6],
                    &v[7], &v[8], &v[9]) != 10)
      continue;
    if (v[9] < 0 || choice_cfg(v[9]) >= kNumCfgs || choice_lg(v[9]) > kMaxSliceLg) continue;
    g_tune_cache[std::make_tuple(v[0], v[1], v[2], v[3], v[4], v[5], v[6], v[7], v[8])] = v[9];
  }
  std::fclose(f);
}

static void append_cache_file_locked(const TuneKey& k, int cfg) {
  if (g_tune_path.empty()) return;
  FILE* f = std::fopen(g_tune_path.c_str(), "a");
  if (!f) return;
  std::fprintf(f, "%d %d %d %d %d %d %d %d %d -> %d\n", std::get<0>(k), std::get<1>(k), std::get<2>(k),
               std::get<3>(k), std::get<4>(k), std::get<5>(k), std::get<6>(k), std::get<7>(k), std::get<8>(k), cfg);
  std::fclose(f);
}

static void append_grouped_line_locked(uint64_t sig, int prec, int cfg) {
  if (g_tune_path.empty()) return;
  FILE* f = std::fopen(g_tune_path.c_str(), "a");
  if (!f) return;
  std::fprintf(f, "G %llx %d -> %d\n", (unsigned long long)sig, prec, cfg);
  std::fclose(f);
}

// starting state from TN_TUNE=off|quick|full, TN_TUNE_CACHE=<path>, TN_LOG=1
static void read_env() {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  if (const char* t = std::getenv("TN_TUNE")) {
    if (!std::strcmp(t, "quick") || !std::strcmp(t, "1")) g_tune_level = 1;
    else if (!std::strcmp(t, "full") || !std::strcmp(t, "2")) g_tune_level = 2;
    else g_tune_level = 0;
  }
  if (const char* c = std::getenv("TN_TUNE_CACHE")) {
    g_tune_path = c;
    load_cache_file_locked();
  }
  const char* lg = std::getenv("TN_LOG");
  g_log = lg && lg[0] && std::strcmp(lg, "0") != 0;
}

bool log_enabled() {
  std::call_once(g_env_once, read_env);
  return g_log;
}

int tune_timing_level(hipStream_t st) {
  log_enabled();
  int level;
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    level = g_tune_level;
  }
  if (level == 0 || g_no_timing) return 0;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(st, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return 0;
  return level;
}

int grouped_tune_get(uint64_t sig, int prec) {
  log_enabled();
  std::lock_guard<std::mutex> lk(g_tune_mu);
  auto it = g_grouped_cache.find(std::make_pair(sig, prec));
  return it == g_grouped_cache.end() ? -1 : it->second;
}

void grouped_tune_put(uint64_t sig, int prec, int cfg, bool timed) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_grouped_cache[std::make_pair(sig, prec)] = cfg;
  if (timed) append_grouped_line_locked(sig, prec, cfg);
}

int32_t launch_gemm_cfg(GemmDesc& d, int32_t prec, int cfg, hipStream_t st) {
  if (cfg < 0 || cfg >= kNumCfgs) return fail(TN_ERR_INVALID_ARGUMENT, "bad tile config %d", cfg);
  const Cfg& g = kCfgs[cfg];
  // the problem the kernel runs on (exchanged operands for the swap kinds)
  // and whether the lean kind applies; otherwise the general tile of the
  // same shape runs on the caller's problem
  GemmDesc x = d;
  bool lean = false;
  if (g.split) {
    if (g.swap) {
      GemmDesc e = exchanged(d);
      if (split_ok(e, prec)) {
        x = e;
        lean = true;
      }
    } else {
      lean = split_ok(d, prec);
    }
  }
  const Cfg& t = (g.split && !lean) ? kCfgs[g.fallback] : g;
  const int bm = (lean && g.swap) ? t.bn : t.bm, bn = (lean && g.swap) ? t.bm : t.bn;
  x.tiles_m = (x.M + bm - 1) / bm;
  x.tiles_n = (x.N + bn - 1) / bn;
  const int64_t tiles = (int64_t)x.tiles_m * x.tiles_n;
  if (tiles >= (1ll << 31) || x.batch > 65535) return fail(TN_ERR_UNSUPPORTED, "grid too large");
  hipLaunchKernelGGL(pick_fn(x, prec, cfg, lean), dim3((unsigned)tiles, 1, (unsigned)x.batch),
                     dim3(t.wm * t.wn * t.wk * 64), 0, st, x);
  return hip_check(hipGetLastError(), "gemm launch");
}

static int32_t launch_choice(GemmDesc& d, int32_t prec, int v, hipStream_t st) {
  const int cfg = choice_cfg(v), lg = choice_lg(v);
  if (lg == 0 || !slices_ok(d, lg)) return launch_gemm_cfg(d, prec, cfg, st);
  const int S = 1 << lg;
  GemmDesc x = slice_desc(d, S);
  TN_TRY(launch_gemm_cfg(x, prec, cfg, st));
  const int64_t MN = (int64_t)d.M * d.N;
  hipLaunchKernelGGL(slice_sum_kernel, dim3((unsigned)((MN + 255) / 256)), dim3(256), 0, st, g_splitk, S, d.M, d.N,
                     d.c, d.gm, d.gn, d.a_scale_bits, d.c_absmax);
  return hip_check(hipGetLastError(), "k-slice sum");
}

// tiles of configuration c on the caller's problem
static int64_t cfg_tiles(const GemmDesc& d, int c) {
  const Cfg& g = kCfgs[c];
  return (int64_t)((d.M + g.bm - 1) / g.bm) * ((d.N + g.bn - 1) / g.bn) * d.batch;
}

// the heuristic choice: the estimated tile, cut into k-slices when its tiles
// fill at most half the compute units it can count on (a quarter for four
// slices) and every slice keeps at least 128 of k
static int heuristic_choice(const GemmDesc& d, int prec) {
  const int c = heuristic_cfg(d, prec);
  if (!g_splitk || g_forced_cfg.load() >= 0) return c;
  const int64_t slots = g_shared ? 128 : 256, tiles = cfg_tiles(d, c);
  for (int lg = max_slice_lg(); lg >= 1; --lg)
    if (slices_ok(d, lg) && tiles << lg <= slots && d.K >> lg >= 128) return c + 100 * lg;
  return c;
}

// the stream on which the tuner runs the second copy of a GEMM that shares
// the chip (one per device, default priority, created on first use)
static int32_t twin_stream(hipStream_t& hs) {
  static std::mutex mu;
  static std::vector<hipStream_t> streams;
  int dev = 0;
  TN_TRY(hip_check(hipGetDevice(&dev), "get device"));
  std::lock_guard<std::mutex> lk(mu);
  if ((int)streams.size() <= dev) streams.resize(dev + 1, nullptr);
  if (!streams[dev]) TN_TRY(hip_check(hipStreamCreateWithFlags(&streams[dev], hipStreamNonBlocking), "create stream"));
  hs = streams[dev];
  return TN_OK;
}

// Times every allowed tile on the real operands and returns the fastest.  A
// GEMM that shares the chip is timed as two copies issued together on st
// and on a twin stream, the way the two directions of a sweep overlap: a
// tile that fills the chip alone then queues behind its twin, while one
// that needs half the compute units runs beside it.  Both copies write the
// same values to C (deterministic kernels; |C| maxima are idempotent), and
// the real launch that follows on st overwrites them after the twin is done.
static int tune_cfg(GemmDesc& d, int32_t prec, int level, hipStream_t st) {
  hipStream_t hs = nullptr;
  if (g_shared && twin_stream(hs) != TN_OK) hs = nullptr;
  hipEvent_t e0, e1, ej;
  if (hipEventCreate(&e0) != hipSuccess) return heuristic_cfg(d, prec);
  if (hipEventCreate(&e1) != hipSuccess) {
    hipEventDestroy(e0);
    return heuristic_cfg(d, prec);
  }
  if (hipEventCreateWithFlags(&ej, hipEventDisableTiming) != hipSuccess) {
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    return heuristic_cfg(d, prec);
  }
  int best = heuristic_choice(d, prec);
  float best_ms = 1e30f;
  for (int v = 0; v < kNumCfgs * (max_slice_lg() + 1); ++v) {
    const int c = v % kNumCfgs, lg = v / kNumCfgs;
    const Cfg& g = kCfgs[c];
    if ((int64_t)g.bm * g.bn > 4ll * d.M * d.N && c != 7) continue;  // mostly padding (32 x 32 always runs)
    if (!cfg_allowed(d, prec, c)) continue;
    // k-slices only where the whole GEMM leaves most compute units idle
    if (lg > 0 && (!slices_ok(d, lg) || cfg_tiles(d, c) << lg > 512 || cfg_tiles(d, c) >= 256)) continue;
    const int choice = c + 100 * lg;
    if (launch_choice(d, prec, choice, st) != TN_OK) continue;  // warm-up
    hipEventRecord(e0, st);
    if (hs) hipStreamWaitEvent(hs, e0, 0);
    const int reps = level >= 2 ? 10 : 3;
    for (int r = 0; r < reps; ++r) {
      launch_choice(d, prec, choice, st);
      if (hs) launch_choice(d, prec, choice, hs);
    }
    if (hs) {
      hipEventRecord(ej, hs);
      hipStreamWaitEvent(st, ej, 0);
    }
    hipEventRecord(e1, st);
    hipEventSynchronize(e1);
    float ms = 0.f;
    hipEventElapsedTime(&ms, e0, e1);
    if (ms < best_ms) {
      best_ms = ms;
      best = choice;
    }
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  hipEventDestroy(ej);
  return best;
}

int32_t launch_gemm(GemmDesc& d, int32_t prec, hipStream_t st) {
  const bool log = log_enabled();
  const int forced = g_forced_cfg.load();
  if (forced < 0 && gemm_small_fits(d)) {
    if (log)
      std::fprintf(stderr, "[tn] gemm M=%d N=%d K=%d batch=%d prec=%d -> small-extent path\n", d.M, d.N, d.K,
                   d.batch, (int)prec);
    return launch_gemm_small(d, prec, st);
  }
  int cfg;
  int level;
  // GEMMs sharing the chip are chosen apart: 1000 added to the groups field
  const TuneKey key = std::make_tuple(d.M, d.N, d.K, d.batch, d.a_mode, d.b_mode, d.c_mode, (int)prec,
                                      (int)(d.gm.n * 100 + d.gn.n * 10 + d.gk.n + (g_shared ? 1000 : 0)));
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    level = g_tune_level;
    auto it = g_tune_cache.find(key);
    cfg = it != g_tune_cache.end() ? it->second : -1;
  }
  const char* how = "cached";
  if (forced >= 0) {
    cfg = forced;
    how = "forced";
  } else if (cfg < 0) {
    bool timed = false;
    if (level > 0 && !g_no_timing) {
      hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
      if (hipStreamIsCapturing(st, &cs) == hipSuccess && cs == hipStreamCaptureStatusNone) {
        cfg = tune_cfg(d, prec, level, st);
        timed = true;
      } else {
        cfg = heuristic_choice(d, prec);
      }
    } else {
      cfg = heuristic_choice(d, prec);
    }
    how = timed ? "timed" : "heuristic";
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune_cache[key] = cfg;
    if (timed) append_cache_file_locked(key, cfg);
  }
  const int lg = slices_ok(d, choice_lg(cfg)) ? choice_lg(cfg) : 0;
  if (log) {
    const Cfg& g = kCfgs[choice_cfg(cfg)];
    std::fprintf(stderr,
                 "[tn] gemm M=%d N=%d K=%d batch=%d groups(m,n,k)=(%d,%d,%d) modes(a,b,c)=(%d,%d,%d) prec=%d%s -> "
                 "tile %d (%dx%dx%d, %dx%dx%d waves) x%d k-slices %s\n",
                 d.M, d.N, d.K, d.batch, d.gm.n, d.gn.n, d.gk.n, d.a_mode, d.b_mode, d.c_mode, (int)prec,
                 g_shared ? " shared" : "", choice_cfg(cfg), g.bm, g.bn, g.bk, g.wm, g.wn, g.wk, 1 << lg, how);
  }
  g_last_choice = choice_cfg(cfg);
  return launch_choice(d, prec, choice_cfg(cfg) + 100 * lg, st);
}

// the gather modes the grouped kernel derives for problem p (the same rules)
int grouped_variant(const Gemm2D& p) {
  // the fast m/n-contiguous gathers: whole blocks of four rows, or a partial
  // last one with M >= 4 and a k stride >= 4
  auto fits = [](int m, int64_t sk) { return m % 4 == 0 || (m >= 4 && sk >= 4); };
  const int am = p.sak == 1 ? LOAD_KVEC : (p.sam == 1 && fits(p.M, p.sak)) ? LOAD_MNVEC : LOAD_GENERIC;
  const int bm = p.sbk == 1 ? LOAD_KVEC : (p.sbn == 1 && fits(p.N, p.sbk)) ? LOAD_MNVEC : LOAD_GENERIC;
  if (am == LOAD_GENERIC || bm == LOAD_GENERIC) return 0;
  return 1 + (am == LOAD_MNVEC ? 2 : 0) + (bm == LOAD_MNVEC ? 1 : 0);
}

int32_t launch_gemm_grouped(const Gemm2D* dev_probs, const int32_t* dev_tile_start, int32_t n_probs,
                            int32_t total_tiles, int32_t prec, int cfg, int variant, hipStream_t st) {
  if (n_probs <= 0 || total_tiles <= 0) return TN_OK;
  const Cfg& g = kCfgs[kGroupedCfg[cfg]];
  hipLaunchKernelGGL(pick_grouped(prec, cfg, variant), dim3((unsigned)total_tiles), dim3(g.wm * g.wn * g.wk * 64), 0, st, dev_probs,
                     dev_tile_start, n_probs);
  return hip_check(hipGetLastError(), "grouped gemm launch");
}

}  // namespace tn

extern "C" {

int32_t tn_tune(const char* cache_path, int32_t level) {
  if (level < 0 || level > 2) return tn::fail(TN_ERR_INVALID_ARGUMENT, "tune level %d", level);
  tn::log_enabled();  // the environment's starting state first, so this call overrides it
  std::lock_guard<std::mutex> lk(tn::g_tune_mu);
  if (cache_path) {
    FILE* f = std::fopen(cache_path, "a");
    if (!f) return tn::fail(TN_ERR_DEVICE, "cannot open tile cache %s for appending", cache_path);
    std::fclose(f);
  }
  tn::g_tune_level = level;
  tn::g_tune_cache.clear();
  tn::g_grouped_cache.clear();
  tn::g_tune_path = cache_path ? cache_path : "";
  tn::load_cache_file_locked();
  return TN_OK;
}

int32_t tn_tune_set_level(int32_t level) {
  if (level < 0 || level > 1) return tn::fail(TN_ERR_INVALID_ARGUMENT, "tune level %d", level);
  tn::log_enabled();
  std::lock_guard<std::mutex> lk(tn::g_tune_mu);
  tn::g_tune_level = level;
  tn::g_tune_cache.clear();
  tn::g_grouped_cache.clear();
  tn::load_cache_file_locked();
  return TN_OK;
}

int32_t tn_tune_last_choice(void) { return tn::g_last_choice; }

int32_t tn_tune_force_config(int32_t cfg) {
  if (cfg < -1 || cfg >= tn::kNumCfgs) return tn::fail(TN_ERR_INVALID_ARGUMENT, "tile config %d", cfg);
  tn::g_forced_cfg.store(cfg);
  return TN_OK;
}

int32_t tn_tune_num_configs(void) { return tn::kNumCfgs; }

int32_t tn_tune_force_grouped_config(int32_t cfg) {
  if (cfg < -1 || cfg > 4) return tn::fail(TN_ERR_INVALID_ARGUMENT, "grouped tile config %d", cfg);
  tn::g_forced_grouped.store(cfg);
  return TN_OK;
}
}
