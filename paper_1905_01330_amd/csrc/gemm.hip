// Contraction GEMM: kernel instantiations, tile selection, autotuner and the
// grouped launch used for uneven batches of small problems.
#include <atomic>
#include <chrono>
#include <cstring>
#include <map>
#include <mutex>
#include <tuple>

#include "gemm_inst.h"

namespace tn {

// ---------------------------------------------------------------------------
// tile configurations

struct Cfg {
  int bm, bn, bk, wm, wn;
  float eff;   // relative per-tile efficiency used by the heuristic
  int wk = 1;  // k-slice groups of wm x wn waves
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
};
static constexpr int kNumCfgs = sizeof(kCfgs) / sizeof(kCfgs[0]);

int gemm_num_cfgs() { return kNumCfgs; }

// fast gathers need one merged K axis and vector-friendly layouts on both operands
static int gemm_variant(const GemmDesc& d) {
  if (d.gk.n != 1 || d.a_mode == LOAD_GENERIC || d.b_mode == LOAD_GENERIC || d.a_mode == LOAD_MNSCALAR ||
      d.b_mode == LOAD_MNSCALAR)
    return 0;
  return 1 + (d.a_mode == LOAD_MNVEC ? 2 : 0) + (d.b_mode == LOAD_MNVEC ? 1 : 0);
}

static GemmFn pick_fn(const GemmDesc& d, int prec, int cfg) { return gemm_fn_prec(prec, cfg, gemm_variant(d)); }

// grouped configurations: 0 -> 128x128, 1 -> 64x64, 2 -> 32x32, 3 -> 64x64 in two k-slices
static const int kGroupedCfg[4] = {3, 15, 7, 14};
int grouped_tile_m(int cfg) { return kCfgs[kGroupedCfg[cfg]].bm; }
int grouped_tile_n(int cfg) { return kCfgs[kGroupedCfg[cfg]].bn; }

static GroupedFn pick_grouped(int prec, int cfg, int variant) { return grouped_fn_prec(prec, cfg, variant); }

static int g_forced_cfg = -1;
static std::atomic<int> g_forced_grouped{-1};

int forced_grouped_cfg() { return g_forced_grouped.load(); }

// eight-wave tiles larger than 64 x 64 have a fixed 256-register budget that
// the run-time-mode gathers exceed: they serve the fast gathers only
static bool cfg_allowed(const GemmDesc& d, int c) {
  const Cfg& g = kCfgs[c];
  return g.wm * g.wn * g.wk < 8 || g.bm * g.bn <= 64 * 64 || gemm_variant(d) != 0;
}

static int heuristic_cfg(const GemmDesc& d) {
  if (g_forced_cfg >= 0) return g_forced_cfg;
  constexpr int kSlots = 256;  // one workgroup per compute unit for the large tiles
  double best = 1e300;
  int best_c = 7;   // 32 x 32 tiles fit every problem
  for (int c = 0; c < kNumCfgs; ++c) {
    if (!cfg_allowed(d, c)) continue;
    const Cfg& g = kCfgs[c];
    const int64_t tiles = (int64_t)((d.M + g.bm - 1) / g.bm) * ((d.N + g.bn - 1) / g.bn) * d.batch;
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

static std::mutex g_tune_mu;
static int g_tune_level = 0;
static std::map<std::tuple<int, int, int, int, int, int, int, int, int>, int> g_tune_cache;
static thread_local int g_last_choice = -1;

int32_t launch_gemm_cfg(GemmDesc& d, int32_t prec, int cfg, hipStream_t st) {
  if (cfg < 0 || cfg >= kNumCfgs) return fail(TN_ERR_INVALID_ARGUMENT, "bad tile config %d", cfg);
  const Cfg& g = kCfgs[cfg];
  d.tiles_m = (d.M + g.bm - 1) / g.bm;
  d.tiles_n = (d.N + g.bn - 1) / g.bn;
  const int64_t tiles = (int64_t)d.tiles_m * d.tiles_n;
  if (tiles >= (1ll << 31) || d.batch > 65535) return fail(TN_ERR_UNSUPPORTED, "grid too large");
  hipLaunchKernelGGL(pick_fn(d, prec, cfg), dim3((unsigned)tiles, 1, (unsigned)d.batch), dim3(g.wm * g.wn * g.wk * 64), 0,
                     st, d);
  return hip_check(hipGetLastError(), "gemm launch");
}

static int tune_cfg(GemmDesc& d, int32_t prec, hipStream_t st) {
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return heuristic_cfg(d);
  if (hipEventCreate(&e1) != hipSuccess) {
    hipEventDestroy(e0);
    return heuristic_cfg(d);
  }
  int best = heuristic_cfg(d);
  float best_ms = 1e30f;
  for (int c = 0; c < kNumCfgs; ++c) {
    const Cfg& g = kCfgs[c];
    if ((int64_t)g.bm * g.bn > 4ll * d.M * d.N && c != 7) continue;  // mostly padding (32 x 32 always runs)
    if (!cfg_allowed(d, c)) continue;
    if (launch_gemm_cfg(d, prec, c, st) != TN_OK) continue;  // warm-up
    hipEventRecord(e0, st);
    for (int r = 0; r < 3; ++r) launch_gemm_cfg(d, prec, c, st);
    hipEventRecord(e1, st);
    hipEventSynchronize(e1);
    float ms = 0.f;
    hipEventElapsedTime(&ms, e0, e1);
    if (ms < best_ms) {
      best_ms = ms;
      best = c;
    }
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  return best;
}

int32_t launch_gemm(GemmDesc& d, int32_t prec, hipStream_t st) {
  if (g_forced_cfg < 0 && gemm_small_fits(d)) return launch_gemm_small(d, prec, st);
  int cfg;
  int level;
  auto key = std::make_tuple(d.M, d.N, d.K, d.batch, d.a_mode, d.b_mode, d.c_mode, (int)prec,
                             (int)(d.gm.n * 100 + d.gn.n * 10 + d.gk.n));
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    level = g_tune_level;
    auto it = g_tune_cache.find(key);
    cfg = it != g_tune_cache.end() ? it->second : -1;
  }
  if (g_forced_cfg >= 0) cfg = g_forced_cfg;
  if (cfg < 0) {
    if (level > 0) {
      hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
      if (hipStreamIsCapturing(st, &cs) == hipSuccess && cs == hipStreamCaptureStatusNone)
        cfg = tune_cfg(d, prec, st);
      else
        cfg = heuristic_cfg(d);
    } else {
      cfg = heuristic_cfg(d);
    }
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune_cache[key] = cfg;
  }
  g_last_choice = cfg;
  return launch_gemm_cfg(d, prec, cfg, st);
}

// the gather modes the grouped kernel derives for problem p (the same rules)
int grouped_variant(const Gemm2D& p) {
  auto al = [](const void* q) { return (reinterpret_cast<uintptr_t>(q) & 15) == 0; };
  const int am = (p.sak == 1 && p.K % 4 == 0 && p.sam % 4 == 0 && al(p.a)) ? LOAD_KVEC
               : (p.sam == 1 && p.M % 4 == 0 && p.sak % 4 == 0 && al(p.a)) ? LOAD_MNVEC
                                                                            : LOAD_GENERIC;
  const int bm = (p.sbk == 1 && p.K % 4 == 0 && p.sbn % 4 == 0 && al(p.b)) ? LOAD_KVEC
               : (p.sbn == 1 && p.N % 4 == 0 && p.sbk % 4 == 0 && al(p.b)) ? LOAD_MNVEC
                                                                            : LOAD_GENERIC;
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

int32_t tn_tune_set_level(int32_t level) {
  if (level < 0 || level > 1) return tn::fail(TN_ERR_INVALID_ARGUMENT, "tune level %d", level);
  std::lock_guard<std::mutex> lk(tn::g_tune_mu);
  tn::g_tune_level = level;
  tn::g_tune_cache.clear();
  return TN_OK;
}

int32_t tn_tune_last_choice(void) { return tn::g_last_choice; }

int32_t tn_tune_force_config(int32_t cfg) {
  if (cfg < -1 || cfg >= tn::kNumCfgs) return tn::fail(TN_ERR_INVALID_ARGUMENT, "tile config %d", cfg);
  std::lock_guard<std::mutex> lk(tn::g_tune_mu);
  tn::g_forced_cfg = cfg;
  return TN_OK;
}

int32_t tn_tune_num_configs(void) { return tn::kNumCfgs; }

int32_t tn_tune_force_grouped_config(int32_t cfg) {
  if (cfg < -1 || cfg > 3) return tn::fail(TN_ERR_INVALID_ARGUMENT, "grouped tile config %d", cfg);
  tn::g_forced_grouped.store(cfg);
  return TN_OK;
}
}
