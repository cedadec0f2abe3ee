// Uneven batch of MPS inner products in one call.  Chains of four or more
// sites are contracted from both ends at once (sites 0 .. c-1 from the left,
// n-1 .. c from the right, c = n / 2), so the number of steps is half the
// longest chain.  Every step is two grouped GEMM launches (ket site into the
// environments, then the bra site) over the halves still active: for small
// steps one launch per product over both halves, for larger ones one per
// half and gather variant, the right halves on the caller's stream and the
// left halves on a side stream.  The problems of a launch are described by a
// compact table in the workspace, largest first so the longest tiles start
// earliest.  At the end each chain's two environments meet in an FP64 sum
// over its middle bond.
#include <algorithm>
#include <cstring>
#include <numeric>
#include <vector>

#include "internal.h"

namespace tn {

static size_t align256b(size_t x) { return (x + 255) & ~(size_t)255; }

struct ChainRec {
  float* e[2];        // left environments (in turn)
  float* er[2];       // right environments
  uint32_t* slots;    // left scales: slots[j] for bond j
  uint32_t* rslots;   // right scales: rslots[i] for bond n - i
  int32_t n;          // sites
  int32_t c;          // middle bond: sites 0 .. c-1 from the left, n-1 .. c from the right
  int64_t cnt;        // elements of either environment at bond c
};

__global__ void batched_init_kernel(const ChainRec* chains, int n_chains) {
  const int c = blockIdx.x;
  if (c >= n_chains) return;
  const ChainRec r = chains[c];
  for (int i = threadIdx.x; i <= r.c; i += blockDim.x) r.slots[i] = i == 0 ? 0x3f800000u : 0u;
  for (int i = threadIdx.x; i <= r.n - r.c; i += blockDim.x) r.rslots[i] = i == 0 ? 0x3f800000u : 0u;
  if (threadIdx.x == 0) {
    r.e[0][0] = 1.0f;
    r.er[0][0] = 1.0f;
  }
}

__device__ inline int slot_exponent(uint32_t bits) {
  int e = (int)((bits >> 23) & 0xffu);
  if (e == 0 || e > 253) return 0;
  return e - 127;
}

// one workgroup per chain: sum_{a', a} E_L[a', a] E_R[a', a] at the middle
// bond in FP64 (products of FP32 values are exact), times 2^(the exponents
// applied on both sides), written as a mantissa in [0.5, 1) and a log scale
constexpr int kFinishThreads = 1024;

__global__ void __launch_bounds__(kFinishThreads) batched_finish_kernel(const ChainRec* chains, int n_chains,
                                                                        double* out2) {
  constexpr int NW = kFinishThreads / 64;
  __shared__ double red[2][NW];
  const int c = blockIdx.x;
  if (c >= n_chains) return;
  const ChainRec r = chains[c];
  const float* el = r.e[r.c & 1];
  const float* er = r.er[(r.n - r.c) & 1];
  double v = 0.0, s = 0.0;
  for (int64_t i = threadIdx.x; i < r.cnt; i += kFinishThreads) v += (double)el[i] * (double)er[i];
  for (int i = threadIdx.x; i < r.c; i += kFinishThreads) s += (double)slot_exponent(r.slots[i]);
  for (int i = threadIdx.x; i < r.n - r.c; i += kFinishThreads) s += (double)slot_exponent(r.rslots[i]);
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) {
    v += __shfl_xor(v, o, 64);
    s += __shfl_xor(s, o, 64);
  }
  if ((threadIdx.x & 63) == 0) {
    red[0][threadIdx.x >> 6] = v;
    red[1][threadIdx.x >> 6] = s;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double total = 0.0, ex = 0.0;
#pragma unroll
    for (int w = 0; w < NW; ++w) {
      total += red[0][w];
      ex += red[1][w];
    }
    int e2 = 0;
    const double m = frexp(total, &e2);
    out2[2 * c] = m;
    out2[2 * c + 1] = (ex + (double)e2) * 0.69314718055994530942;
  }
}

namespace {

constexpr int kGroupedCfgs = 5;   // the last (160 x 256, eight waves) for fast-gather launches only
// a step whose problems have no extent above this runs both halves in one
// launch per product (launch latency, not the gathers, sets its time)
constexpr int kSmallStepExtent = 128;

struct Launch {
  size_t prob_off;                   // index into the problem table
  int32_t n_probs;
  size_t tile_off[kGroupedCfgs];     // per grouped tile: index into the tile-start table
  int32_t tiles[kGroupedCfgs];       // per grouped tile: workgroups of the launch
  int heur;                          // the tile the work estimate picks
  int variant;                       // gather variant shared by every problem of the launch
  int side;                          // 0: the caller's stream (right halves), 1: the side stream (left halves)
  bool has_left;                     // a caller's-stream launch that holds left halves too (small steps)
  uint64_t sig;                      // the step's problems (shapes and variant), for the tile cache
};

struct BatchPlan {
  std::vector<ChainRec> chains;
  std::vector<Gemm2D> probs;
  std::vector<int32_t> tstart;
  std::vector<Launch> launches;
  size_t chain_bytes = 0, chain_tab = 0, prob_tab = 0, tile_tab = 0, total = 0;
};

bool is_contiguous(const tn_tensor& t) {
  int64_t st = 1;
  for (int k = t.rank - 1; k >= 0; --k) {
    if (t.shape[k] > 1 && t.stride[k] != st) return false;
    st *= t.shape[k];
  }
  return true;
}

// Work estimate of the tile for one site step, shared by all of its problems
// (one launch per step, product and half); used when tuning is off or the stream
// is being captured.  With tuning on, the first launch of each step
// signature and precision times the grouped tiles instead.  A step is usually too small to fill the chip with
// 128 x 128 tiles, so its time is the latency of one tile rather than the
// total work: the estimate is, in units of one wave's 32 x 32 block times one
// k, the larger of the longest wave's work and the total padded work spread
// over the 1024 SIMDs, divided by a per-wave efficiency of the tile shape.
// The efficiencies follow per-launch measurement on a batch of 32 chains
// with odd bond dimensions (run-time gathers; N up to 256, chi up to 512):
// the 128 x 128 tile was 10-25 % faster on the full steps, the k-sliced
// 64 x 64 tile about twice as fast on the last steps, where few tiles run.
//   0: 128 x 128 (four 64 x 64 waves)   1: 64 x 64 (four 32 x 32 waves)
//   3: 64 x 64 in two k-slices (eight waves, each over half of K)
//   2: 32 x 32 when every problem of the step fits one such tile
// chains of at least this many sites are contracted from both ends
constexpr int kTwoSided = 4;

int step_cfg(const std::vector<Gemm2D>& v) {
  bool tiny = true;
  for (const Gemm2D& q : v) tiny = tiny && q.M <= 32 && q.N <= 32;
  if (tiny) return 2;
  struct Cand {
    int cfg, bm;
    double per_wave;  // blocks x k per wave, per k of the problem
    double eff;
  };
  static const Cand cands[] = {{0, 128, 4.0, 1.2}, {1, 64, 1.0, 0.9}, {3, 64, 0.5, 1.0}};
  int best = 0;
  double best_t = 1e300;
  for (const Cand& c : cands) {
    double work = 0, lat = 0;
    for (const Gemm2D& q : v) {
      const double tiles = (double)((q.M + c.bm - 1) / c.bm) * ((q.N + c.bm - 1) / c.bm);
      work += tiles * (c.bm / 32) * (c.bm / 32) * q.K;
      lat = std::max(lat, c.per_wave * q.K);
    }
    const double t = std::max(lat, work / 1024.0) / c.eff;
    if (t < best_t * 0.999) {
      best_t = t;
      best = c.cfg;
    }
  }
  return best;
}

static int32_t add_launch(BatchPlan& P, std::vector<std::pair<int64_t, Gemm2D>>& u, int var, int side, bool has_left);

int32_t build(int32_t n_chains, const int32_t* off, const tn_tensor* psi, const tn_tensor* phi, char* ws,
              BatchPlan& P) {
  if (n_chains < 1) return fail(TN_ERR_INVALID_ARGUMENT, "n_chains must be >= 1");
  if (!off || !psi || !phi) return fail(TN_ERR_INVALID_ARGUMENT, "NULL chain description");
  if (off[0] != 0) return fail(TN_ERR_INVALID_ARGUMENT, "site_offsets[0] must be 0");
  std::vector<std::vector<int64_t>> dp(n_chains), dq(n_chains);
  std::vector<int64_t> phys(n_chains);
  std::vector<size_t> ebytes(n_chains), tbytes(n_chains);
  size_t chain_total = 0;
  for (int c = 0; c < n_chains; ++c) {
    const int n = off[c + 1] - off[c];
    if (n < 1) return fail(TN_ERR_INVALID_ARGUMENT, "chain %d has no sites", c);
    for (int k = 0; k < n; ++k) {
      const tn_tensor& a = psi[off[c] + k];
      const tn_tensor& b = phi[off[c] + k];
      TN_TRY(check_tensor(&a, "psi_sites[i]", TN_F32));
      TN_TRY(check_tensor(&b, "phi_sites[i]", TN_F32));
      if (a.rank != 3 || b.rank != 3) return fail(TN_ERR_SHAPE_MISMATCH, "chain %d site %d: sites must be rank 3", c, k);
      if (!is_contiguous(a) || !is_contiguous(b))
        return fail(TN_ERR_UNSUPPORTED, "chain %d site %d: batched sites must be contiguous", c, k);
      if (k == 0) {
        if (a.shape[0] != 1 || b.shape[0] != 1) return fail(TN_ERR_SHAPE_MISMATCH, "chain %d: first bond must be 1", c);
        phys[c] = a.shape[1];
        dp[c].push_back(1);
        dq[c].push_back(1);
      } else if (a.shape[0] != dp[c].back() || b.shape[0] != dq[c].back()) {
        return fail(TN_ERR_SHAPE_MISMATCH, "chain %d: bond %d does not match", c, k);
      }
      if (a.shape[1] != phys[c] || b.shape[1] != phys[c])
        return fail(TN_ERR_SHAPE_MISMATCH, "chain %d site %d: physical dimensions differ", c, k);
      dp[c].push_back(a.shape[2]);
      dq[c].push_back(b.shape[2]);
    }
    if (dp[c].back() != 1 || dq[c].back() != 1) return fail(TN_ERR_SHAPE_MISMATCH, "chain %d: last bond must be 1", c);
    int64_t me = 1, mt = 1;
    for (int k = 0; k <= n; ++k) me = std::max(me, dp[c][k] * dq[c][k]);
    for (int k = 0; k < n; ++k) mt = std::max(mt, dp[c][k] * phys[c] * dq[c][k + 1]);
    ebytes[c] = align256b(me * 4);
    tbytes[c] = align256b(mt * 4);
    chain_total += 4 * ebytes[c] + 2 * tbytes[c] + 2 * align256b((size_t)(n + 1) * 4);
  }
  // problem tables
  std::vector<int> order(n_chains);
  std::iota(order.begin(), order.end(), 0);
  P.chains.resize(n_chains);
  size_t o = 0;
  std::vector<float*> tbuf(n_chains), trbuf(n_chains);
  int max_steps = 0;
  for (int c = 0; c < n_chains; ++c) {
    ChainRec& r = P.chains[c];
    for (int h = 0; h < 2; ++h) {
      r.e[h] = reinterpret_cast<float*>(ws + o);
      o += ebytes[c];
    }
    for (int h = 0; h < 2; ++h) {
      r.er[h] = reinterpret_cast<float*>(ws + o);
      o += ebytes[c];
    }
    tbuf[c] = reinterpret_cast<float*>(ws + o);
    o += tbytes[c];
    trbuf[c] = reinterpret_cast<float*>(ws + o);
    o += tbytes[c];
    r.n = off[c + 1] - off[c];
    r.c = r.n < kTwoSided ? r.n : r.n / 2;
    r.cnt = dp[c][r.c] * dq[c][r.c];
    r.slots = reinterpret_cast<uint32_t*>(ws + o);
    o += align256b((size_t)(r.n + 1) * 4);
    r.rslots = reinterpret_cast<uint32_t*>(ws + o);
    o += align256b((size_t)(r.n + 1) * 4);
    max_steps = std::max(max_steps, std::max(r.c, r.n - r.c));
  }
  P.chain_bytes = o;
  for (int j = 0; j < max_steps; ++j) {
    std::vector<std::pair<int64_t, Gemm2D>> vs[2], vls[2];   // per product: right halves, left halves
    for (int g = 0; g < 2; ++g) {
      std::vector<std::pair<int64_t, Gemm2D>>& v = vs[g];
      std::vector<std::pair<int64_t, Gemm2D>>& vl = vls[g];
      for (int c = 0; c < n_chains; ++c) {
        const ChainRec& r = P.chains[c];
        if (j >= r.n - r.c) continue;
        // right half: site k = n-1-j, E_R at bond k+1 in er[j & 1]
        const int k = r.n - 1 - j;
        const tn_tensor& a = psi[off[c] + k];
        const tn_tensor& b = phi[off[c] + k];
        const int64_t da = dp[c][k], da2 = dp[c][k + 1], d = phys[c], db = dq[c][k], db2 = dq[c][k + 1];
        Gemm2D q;
        std::memset(&q, 0, sizeof(q));
        if (g == 0) {  // T[(a' s), b] = sum_b' psi[(a' s), b'] E_R[b', b]  (scaled by 2^-e: exact)
          q.a = static_cast<const float*>(a.data);
          q.b = r.er[j & 1];
          q.c = trbuf[c];
          q.M = (int32_t)(da * d);
          q.K = (int32_t)da2;
          q.N = (int32_t)db2;
          q.sam = da2;
          q.sak = 1;
          q.sbk = db2;
          q.sbn = 1;
          q.scm = db2;
          q.scn = 1;
          q.a_scale_bits = r.rslots + j;
        } else {  // E_R'[a', a] = sum_{(s b)} T[a', (s b)] phi[a, (s b)]
          q.a = trbuf[c];
          q.b = static_cast<const float*>(b.data);
          q.c = r.er[(j + 1) & 1];
          q.M = (int32_t)da;
          q.K = (int32_t)(d * db2);
          q.N = (int32_t)db;
          q.sam = d * db2;
          q.sak = 1;
          q.sbk = 1;
          q.sbn = d * db2;
          q.scm = db;
          q.scn = 1;
          q.c_absmax = r.rslots + j + 1;
        }
        v.push_back({(int64_t)q.M * q.N * q.K, q});
      }
      for (int c = 0; c < n_chains; ++c) {
        if (j >= P.chains[c].c) continue;
        const tn_tensor& a = psi[off[c] + j];
        const tn_tensor& b = phi[off[c] + j];
        const int64_t pa = dp[c][j], qa = dq[c][j], d = phys[c], pb = dp[c][j + 1], qb = dq[c][j + 1];
        ChainRec& r = P.chains[c];
        Gemm2D q;
        std::memset(&q, 0, sizeof(q));
        if (g == 0) {  // T[a', (s b)] = sum_a E[a', a] phi[a, (s b)]
          q.a = r.e[j & 1];
          q.b = static_cast<const float*>(b.data);
          q.c = tbuf[c];
          q.M = (int32_t)pa;
          q.K = (int32_t)qa;
          q.N = (int32_t)(d * qb);
          q.sam = qa;
          q.sak = 1;
          q.sbk = d * qb;
          q.sbn = 1;
          q.scm = d * qb;
          q.scn = 1;
          q.a_scale_bits = r.slots + j;
        } else {  // E'[b', b] = sum_{(a' s)} psi[(a' s), b'] T[(a' s), b]
          q.a = static_cast<const float*>(a.data);
          q.b = tbuf[c];
          q.c = r.e[(j + 1) & 1];
          q.M = (int32_t)pb;
          q.K = (int32_t)(pa * d);
          q.N = (int32_t)qb;
          q.sam = 1;
          q.sak = pb;
          q.sbk = qb;
          q.sbn = 1;
          q.scm = qb;
          q.scn = 1;
          q.c_absmax = r.slots + j + 1;
        }
        vl.push_back({(int64_t)q.M * q.N * q.K, q});
      }
    }
    // A step whose extents are all small is bound by launch latency: both
    // halves go into one launch per product on the caller's stream (the
    // run-time gathers when their layouts differ).  In a larger step the
    // right halves run on the caller's stream and the left halves on a side
    // stream, the halves being independent until the final sums; their
    // products have different layouts (a left bra product reads both
    // operands along their rows), so each launch holds one half and one
    // gather variant and takes the fast gathers.  The largest problems of a
    // launch take the first tiles.
    bool small = true;
    for (int g = 0; g < 2; ++g)
      for (const auto* w : {&vs[g], &vls[g]})
        for (const auto& e : *w)
          if (std::max(e.second.M, std::max(e.second.N, e.second.K)) > kSmallStepExtent) small = false;
    for (int g = 0; g < 2; ++g) {
      if (small) {
        std::vector<std::pair<int64_t, Gemm2D>> u = vs[g];
        u.insert(u.end(), vls[g].begin(), vls[g].end());
        if (u.empty()) continue;
        int var = grouped_variant(u[0].second);
        for (const auto& e : u)
          if (grouped_variant(e.second) != var) var = 0;
        TN_TRY(add_launch(P, u, var, 0, !vls[g].empty()));
        continue;
      }
      for (int side = 0; side < 2; ++side)
        for (int var = 0; var <= 4; ++var) {
          std::vector<std::pair<int64_t, Gemm2D>> u;
          for (auto& e : side == 0 ? vs[g] : vls[g])
            if (grouped_variant(e.second) == var) u.push_back(e);
          if (u.empty()) continue;
          TN_TRY(add_launch(P, u, var, side, false));
        }
    }
  }
  P.chain_tab = align256b(P.chain_bytes);
  P.prob_tab = P.chain_tab + align256b(P.chains.size() * sizeof(ChainRec));
  P.tile_tab = P.prob_tab + align256b(P.probs.size() * sizeof(Gemm2D));
  P.total = P.tile_tab + align256b(P.tstart.size() * sizeof(int32_t));
  return TN_OK;
}

// one grouped launch over problems u (one half, one gather variant)
static int32_t add_launch(BatchPlan& P, std::vector<std::pair<int64_t, Gemm2D>>& u, int var, int side, bool has_left) {
  std::stable_sort(u.begin(), u.end(), [](const auto& x, const auto& y) { return x.first > y.first; });
  std::vector<Gemm2D> qs;
  for (auto& e : u) qs.push_back(e.second);
  Launch L;
  L.prob_off = P.probs.size();
  L.n_probs = (int32_t)u.size();
  L.heur = step_cfg(qs);
  L.variant = var;
  L.side = side;
  L.has_left = has_left;
  // FNV-1a over the problem shapes in launch order, the variant and the half
  uint64_t h = 1469598103934665603ull;
  auto mix = [&h](uint64_t x) {
    for (int b = 0; b < 8; ++b) {
      h ^= (x >> (8 * b)) & 0xffu;
      h *= 1099511628211ull;
    }
  };
  mix((uint64_t)var);
  mix((uint64_t)side);
  for (const Gemm2D& q : qs) {
    mix((uint64_t)q.M);
    mix((uint64_t)q.N);
    mix((uint64_t)q.K);
    P.probs.push_back(q);
  }
  L.sig = h;
  // a tile-start table for every grouped tile, so the tile can be chosen per launch
  for (int g2 = 0; g2 < kGroupedCfgs; ++g2) {
    const int tm = grouped_tile_m(g2), tn_ = grouped_tile_n(g2);
    L.tile_off[g2] = P.tstart.size();
    int64_t t = 0;
    for (const Gemm2D& q : qs) {
      P.tstart.push_back((int32_t)t);
      t += (int64_t)((q.M + tm - 1) / tm) * ((q.N + tn_ - 1) / tn_);
    }
    if (t >= (1ll << 31)) return fail(TN_ERR_UNSUPPORTED, "too many tiles in one step");
    L.tiles[g2] = (int32_t)t;
  }
  P.launches.push_back(L);
  return TN_OK;
}

}  // namespace

}  // namespace tn

using namespace tn;

extern "C" {

int32_t tn_mps_inner_batched_workspace(int32_t n_chains, const int32_t* site_offsets, const tn_tensor* psi_sites,
                                       const tn_tensor* phi_sites, size_t* bytes) {
  if (!bytes) return fail(TN_ERR_INVALID_ARGUMENT, "bytes is NULL");
  BatchPlan P;
  TN_TRY(build(n_chains, site_offsets, psi_sites, phi_sites, nullptr, P));
  *bytes = P.total;
  return TN_OK;
}

int32_t tn_mps_inner_batched_upload(int32_t n_chains, const int32_t* site_offsets, const tn_tensor* psi_sites,
                                    const tn_tensor* phi_sites, void* workspace, size_t ws_bytes, void* stream) {
  BatchPlan P;
  TN_TRY(build(n_chains, site_offsets, psi_sites, phi_sites, nullptr, P));
  if (ws_bytes < P.total || !workspace) return fail(TN_ERR_WORKSPACE_TOO_SMALL, "workspace needs %zu bytes", P.total);
  BatchPlan Q;
  char* ws = static_cast<char*>(workspace);
  TN_TRY(build(n_chains, site_offsets, psi_sites, phi_sites, ws, Q));
  hipStream_t st = static_cast<hipStream_t>(stream);
  TN_TRY(hip_check(hipMemcpyAsync(ws + Q.chain_tab, Q.chains.data(), Q.chains.size() * sizeof(ChainRec),
                                  hipMemcpyHostToDevice, st),
                   "chain table upload"));
  TN_TRY(hip_check(hipMemcpyAsync(ws + Q.prob_tab, Q.probs.data(), Q.probs.size() * sizeof(Gemm2D), hipMemcpyHostToDevice, st),
                   "problem table upload"));
  TN_TRY(hip_check(hipMemcpyAsync(ws + Q.tile_tab, Q.tstart.data(), Q.tstart.size() * sizeof(int32_t),
                                  hipMemcpyHostToDevice, st),
                   "tile table upload"));
  // the host tables are released when this call returns
  return hip_check(hipStreamSynchronize(st), "table upload");
}

int32_t tn_mps_inner_batched_launch(int32_t n_chains, const int32_t* site_offsets, const tn_tensor* psi_sites,
                                    const tn_tensor* phi_sites, double* out2, void* workspace, size_t ws_bytes,
                                    int32_t prec, void* stream) {
  if (!out2) return fail(TN_ERR_INVALID_ARGUMENT, "out2 is NULL");
  if (prec < 0 || prec > 3) return fail(TN_ERR_UNSUPPORTED, "unknown precision %d", prec);
  BatchPlan P;
  TN_TRY(build(n_chains, site_offsets, psi_sites, phi_sites, nullptr, P));
  if (ws_bytes < P.total || !workspace) return fail(TN_ERR_WORKSPACE_TOO_SMALL, "workspace needs %zu bytes", P.total);
  // the host-side launch list is rebuilt (no device work); the tables are the upload's
  BatchPlan Q;
  char* ws = static_cast<char*>(workspace);
  TN_TRY(build(n_chains, site_offsets, psi_sites, phi_sites, ws, Q));
  hipStream_t st = static_cast<hipStream_t>(stream);
  ChainRec* d_chains = reinterpret_cast<ChainRec*>(ws + Q.chain_tab);
  Gemm2D* d_probs = reinterpret_cast<Gemm2D*>(ws + Q.prob_tab);
  int32_t* d_tiles = reinterpret_cast<int32_t*>(ws + Q.tile_tab);
  hipLaunchKernelGGL(batched_init_kernel, dim3(n_chains), dim3(64), 0, st, d_chains, n_chains);
  TN_TRY(hip_check(hipGetLastError(), "batched init"));
  const int forced = forced_grouped_cfg();
  const int level = forced >= 0 ? 0 : tune_timing_level(st);
  // the left halves of the larger steps run on a side stream: the work
  // moves to it (an event on `stream` it waits for) at the first such
  // launch and back (an event on it that `stream` waits for) before a
  // launch that holds left halves on `stream`, and before the sums
  // (capturable)
  hipStream_t ls = st;
  TN_TRY(side_stream(ls));
  hipEvent_t hop = nullptr;
  TN_TRY(hip_check(hipEventCreateWithFlags(&hop, hipEventDisableTiming), "create event"));
  bool left_on_side = false;
  auto run = [&](const Launch& L, int cfg, hipStream_t s) {
    return launch_gemm_grouped(d_probs + L.prob_off, d_tiles + L.tile_off[cfg], L.n_probs, L.tiles[cfg], prec, cfg,
                               L.variant, s);
  };
  hipEvent_t e0 = nullptr, e1 = nullptr;
  auto issue = [&](const Launch& L) -> int32_t {
    const hipStream_t s = L.side ? ls : st;
    // the eight-wave tile serves fast-gather launches only
    const int ncfg = L.variant ? kGroupedCfgs : kGroupedCfgs - 1;
    int cfg = forced >= 0 ? (forced < ncfg ? forced : 0) : grouped_tune_get(L.sig, prec);
    if (cfg >= ncfg) cfg = 0;
    if (cfg < 0) {
      bool timed = false;
      cfg = L.heur;
      if (level > 0) {
        // time every grouped tile on this step, with the step's real
        // inputs (a launch only writes its own outputs, so repeating it
        // recomputes the same values), and keep the fastest
        if (!e0) {
          TN_TRY(hip_check(hipEventCreate(&e0), "tuning event"));
          TN_TRY(hip_check(hipEventCreate(&e1), "tuning event"));
        }
        float best = 1e30f;
        const int reps = level >= 2 ? 10 : 3;
        for (int c = 0; c < ncfg; ++c) {
          TN_TRY(run(L, c, s));
          TN_TRY(hip_check(hipEventRecord(e0, s), "tuning event"));
          for (int r = 0; r < reps; ++r) TN_TRY(run(L, c, s));
          TN_TRY(hip_check(hipEventRecord(e1, s), "tuning event"));
          TN_TRY(hip_check(hipEventSynchronize(e1), "tuning event"));
          float ms = 0.f;
          TN_TRY(hip_check(hipEventElapsedTime(&ms, e0, e1), "tuning event"));
          if (ms < best) {
            best = ms;
            cfg = c;
          }
        }
        timed = true;
      }
      grouped_tune_put(L.sig, prec, cfg, timed);
    }
    return run(L, cfg, s);
  };
  int32_t rc = TN_OK;
  for (const Launch& L : Q.launches) {
    if (L.side == 1 && !left_on_side) {
      hipEventRecord(hop, st);
      hipStreamWaitEvent(ls, hop, 0);
      left_on_side = true;
    } else if (L.side == 0 && L.has_left && left_on_side) {
      hipEventRecord(hop, ls);
      hipStreamWaitEvent(st, hop, 0);
      left_on_side = false;
    }
    rc = issue(L);
    if (rc != TN_OK) break;
  }
  if (e0) hipEventDestroy(e0);
  if (e1) hipEventDestroy(e1);
  if (left_on_side) {
    hipEventRecord(hop, ls);
    hipStreamWaitEvent(st, hop, 0);
  }
  hipEventDestroy(hop);
  TN_TRY(rc);
  hipLaunchKernelGGL(batched_finish_kernel, dim3(n_chains), dim3(kFinishThreads), 0, st, d_chains, n_chains, out2);
  return hip_check(hipGetLastError(), "batched finish");
}

int32_t tn_mps_inner_batched(int32_t n_chains, const int32_t* site_offsets, const tn_tensor* psi_sites,
                             const tn_tensor* phi_sites, double* out2, void* workspace, size_t ws_bytes, int32_t prec,
                             void* stream) {
  if (!out2) return fail(TN_ERR_INVALID_ARGUMENT, "out2 is NULL");
  if (prec < 0 || prec > 3) return fail(TN_ERR_UNSUPPORTED, "unknown precision %d", prec);
  TN_TRY(tn_mps_inner_batched_upload(n_chains, site_offsets, psi_sites, phi_sites, workspace, ws_bytes, stream));
  return tn_mps_inner_batched_launch(n_chains, site_offsets, psi_sites, phi_sites, out2, workspace, ws_bytes, prec,
                                     stream);
}

}  // extern "C"
