// ncon network driver (Appendix B): validates the label lists, simulates the
// contraction sequence on the host, then runs one trace / pairwise
// contraction / outer product per step.  Intermediates are carved from the
// caller's workspace; the last step stores straight into the caller's output
// through a permuted view (the final reorder of the dangling edges).
#include <algorithm>
#include <cstring>
#include <map>
#include <mutex>
#include <vector>

#include "internal.h"

namespace tn {

namespace {

struct Node {
  std::vector<int32_t> labels;
  std::vector<int64_t> shape;
  int input;        // >= 0: caller's node index; -1: intermediate
  size_t ws_off;    // intermediate: byte offset in the workspace
  std::vector<int> mem;   // intermediate: axes from outermost to innermost in memory (empty: as listed)
};

// element strides of an intermediate laid out in `mem` order
std::vector<int64_t> mem_strides(const Node& n) {
  const int r = (int)n.shape.size();
  std::vector<int64_t> st(r, 1);
  if (n.mem.empty()) {
    for (int a = r - 2; a >= 0; --a) st[a] = st[a + 1] * n.shape[a + 1];
    return st;
  }
  int64_t acc = 1;
  for (int i = r - 1; i >= 0; --i) {
    st[n.mem[i]] = acc;
    acc *= n.shape[n.mem[i]];
  }
  return st;
}

enum StepKind { STEP_TRACE, STEP_CONTRACT, STEP_OUTER, STEP_COPY };

struct Step {
  StepKind kind;
  int x, y;                   // node ids (y unused for trace/copy)
  std::vector<int32_t> ax, bx;  // trace axes (ax[0], ax[1]) or contracted pairs
  int result;                 // node id
};

struct Plan {
  std::vector<Node> nodes;
  std::vector<Step> steps;
  size_t ws_bytes = 0;
  size_t scratch_off = 0;   // reduction scratch: byte offset in the workspace
  size_t slices_off = 0;    // k-slice partial results: byte offset, floats
  size_t slices_floats = 0;
  int final_node = -1;
};

// k-slices of a network step: up to 64 (a contraction whose result is a few
// tiles and whose contracted extent is long runs on 64x the workgroups),
// their partial results capped at 16 MiB
constexpr int kNetSliceLg = 6;
constexpr size_t kNetSliceCapFloats = size_t(1) << 22;

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

int32_t build_plan(int32_t n_nodes, const tn_tensor* nodes, const int32_t* labels, const int32_t* offsets,
                   int32_t n_order, const int32_t* order, Plan& plan) {
  if (n_nodes < 1) return fail(TN_ERR_INVALID_ARGUMENT, "network needs at least one node");
  if (!nodes || !labels || !offsets) return fail(TN_ERR_INVALID_ARGUMENT, "NULL network description");
  if (offsets[0] != 0) return fail(TN_ERR_INVALID_ARGUMENT, "offsets[0] must be 0");
  std::map<int32_t, std::vector<std::pair<int, int>>> where;  // label -> (node, axis)
  for (int i = 0; i < n_nodes; ++i) {
    char nm[32];
    snprintf(nm, sizeof(nm), "nodes[%d]", i);
    TN_TRY(check_tensor(&nodes[i], nm, TN_F32));
    if (offsets[i + 1] - offsets[i] != nodes[i].rank)
      return fail(TN_ERR_INVALID_ARGUMENT, "node %d: %d labels for rank %d", i, offsets[i + 1] - offsets[i], nodes[i].rank);
    Node n;
    n.input = i;
    n.ws_off = 0;
    for (int a = 0; a < nodes[i].rank; ++a) {
      int32_t l = labels[offsets[i] + a];
      n.labels.push_back(l);
      n.shape.push_back(nodes[i].shape[a]);
      where[l].push_back({i, a});
    }
    plan.nodes.push_back(n);
  }
  int n_open = 0;
  std::vector<int32_t> closed;
  for (auto& kv : where) {
    if (kv.first >= 0) {
      if (kv.second.size() != 2) return fail(TN_ERR_INVALID_ARGUMENT, "label %d appears %zu times", kv.first, kv.second.size());
      auto p = kv.second[0], q = kv.second[1];
      if (nodes[p.first].shape[p.second] != nodes[q.first].shape[q.second])
        return fail(TN_ERR_SHAPE_MISMATCH, "label %d joins axes of different extent", kv.first);
      closed.push_back(kv.first);
    } else {
      if (kv.second.size() != 1) return fail(TN_ERR_INVALID_ARGUMENT, "open label %d repeated", kv.first);
      ++n_open;
    }
  }
  for (int q = 1; q <= n_open; ++q)
    if (!where.count(-q)) return fail(TN_ERR_INVALID_ARGUMENT, "open labels must be -1..-%d", n_open);
  std::vector<int32_t> seq;
  if (n_order > 0 && order) {
    std::vector<int32_t> chk(order, order + n_order);
    std::vector<int32_t> srt = chk;
    std::sort(srt.begin(), srt.end());
    if (srt != closed) return fail(TN_ERR_INVALID_ARGUMENT, "order must list every connected label once");
    seq = chk;
  } else {
    seq = closed;
  }

  std::vector<int> alive;
  for (int i = 0; i < n_nodes; ++i) alive.push_back(i);
  auto new_node = [&](std::vector<int32_t> l, std::vector<int64_t> s) {
    Node n;
    n.labels = std::move(l);
    n.shape = std::move(s);
    n.input = -1;
    n.ws_off = 0;
    plan.nodes.push_back(n);
    return (int)plan.nodes.size() - 1;
  };
  std::map<int32_t, bool> done;
  for (int32_t lab : seq) {
    if (done[lab]) continue;
    std::vector<int> hold;
    for (int id : alive) {
      auto& L = plan.nodes[id].labels;
      if (std::find(L.begin(), L.end(), lab) != L.end()) hold.push_back(id);
    }
    if (hold.size() == 1) {
      Node& n = plan.nodes[hold[0]];
      std::vector<int32_t> ax;
      for (int a = 0; a < (int)n.labels.size(); ++a)
        if (n.labels[a] == lab) ax.push_back(a);
      std::vector<int32_t> nl;
      std::vector<int64_t> ns;
      for (int a = 0; a < (int)n.labels.size(); ++a)
        if (n.labels[a] != lab) {
          nl.push_back(n.labels[a]);
          ns.push_back(n.shape[a]);
        }
      int x = hold[0];
      int r = new_node(nl, ns);
      Step st;
      st.kind = STEP_TRACE;
      st.x = x;
      st.y = -1;
      st.ax = ax;
      st.result = r;
      plan.steps.push_back(st);
      *std::find(alive.begin(), alive.end(), x) = r;
      done[lab] = true;
      continue;
    }
    int x = hold[0], y = hold[1];
    const Node nx = plan.nodes[x], ny = plan.nodes[y];
    Step st;
    st.kind = STEP_CONTRACT;
    st.x = x;
    st.y = y;
    std::vector<bool> cx(nx.labels.size(), false), cy(ny.labels.size(), false);
    for (int a = 0; a < (int)nx.labels.size(); ++a) {
      int32_t l = nx.labels[a];
      if (l < 0) continue;
      for (int b = 0; b < (int)ny.labels.size(); ++b)
        if (ny.labels[b] == l && !cy[b]) {
          st.ax.push_back(a);
          st.bx.push_back(b);
          cx[a] = cy[b] = true;
          done[l] = true;
          break;
        }
    }
    std::vector<int32_t> nl;
    std::vector<int64_t> ns;
    for (int a = 0; a < (int)nx.labels.size(); ++a)
      if (!cx[a]) {
        nl.push_back(nx.labels[a]);
        ns.push_back(nx.shape[a]);
      }
    for (int b = 0; b < (int)ny.labels.size(); ++b)
      if (!cy[b]) {
        nl.push_back(ny.labels[b]);
        ns.push_back(ny.shape[b]);
      }
    if ((int)nl.size() > TN_MAX_RANK) return fail(TN_ERR_UNSUPPORTED, "intermediate rank %zu exceeds %d", nl.size(), TN_MAX_RANK);
    st.result = new_node(nl, ns);
    plan.steps.push_back(st);
    alive.erase(std::find(alive.begin(), alive.end(), x));
    alive.erase(std::find(alive.begin(), alive.end(), y));
    alive.push_back(st.result);
  }
  // disconnected pieces: outer products in list order
  while (alive.size() > 1) {
    int x = alive[0], y = alive[1];
    std::vector<int32_t> nl = plan.nodes[x].labels;
    std::vector<int64_t> ns = plan.nodes[x].shape;
    nl.insert(nl.end(), plan.nodes[y].labels.begin(), plan.nodes[y].labels.end());
    ns.insert(ns.end(), plan.nodes[y].shape.begin(), plan.nodes[y].shape.end());
    if ((int)nl.size() > TN_MAX_RANK) return fail(TN_ERR_UNSUPPORTED, "outer product rank exceeds %d", TN_MAX_RANK);
    Step st;
    st.kind = STEP_OUTER;
    st.x = x;
    st.y = y;
    st.result = new_node(nl, ns);
    plan.steps.push_back(st);
    alive.erase(alive.begin(), alive.begin() + 2);
    alive.insert(alive.begin(), st.result);
  }
  if (plan.steps.empty()) {
    Step st;
    st.kind = STEP_COPY;
    st.x = alive[0];
    st.y = -1;
    st.result = new_node(plan.nodes[alive[0]].labels, plan.nodes[alive[0]].shape);
    plan.steps.push_back(st);
  }
  plan.final_node = plan.steps.back().result;
  // Memory order of the intermediates that feed a pairwise contraction: the
  // axes contracted in that step form one block, outermost, in the order of
  // the partner's strides (so the contracted index merges into one strided
  // axis in both operands and the GEMM takes its fast gathers), and the
  // other axes follow in their listed order (the producer's last free axis
  // stays innermost, so its stores stay contiguous).  The stores of every
  // step go through the output's strides, so any order costs nothing there.
  auto strides_of = [&](int id) -> std::vector<int64_t> {
    const Node& n = plan.nodes[id];
    if (n.input >= 0) return std::vector<int64_t>(nodes[n.input].stride, nodes[n.input].stride + n.shape.size());
    return mem_strides(n);
  };
  std::vector<bool> decided(plan.nodes.size(), false);
  auto arrange = [&](int id, const std::vector<int32_t>& own, int partner, const std::vector<int32_t>& theirs) {
    Node& n = plan.nodes[id];
    if (n.input >= 0 || id == plan.final_node || decided[id]) return;
    const std::vector<int64_t> ps = strides_of(partner);
    std::vector<int> idx(own.size());
    for (size_t i = 0; i < idx.size(); ++i) idx[i] = (int)i;
    std::stable_sort(idx.begin(), idx.end(), [&](int p, int q) { return ps[theirs[p]] > ps[theirs[q]]; });
    std::vector<bool> used(n.shape.size(), false);
    n.mem.clear();
    for (int i : idx) {
      n.mem.push_back(own[i]);
      used[own[i]] = true;
    }
    for (int a = 0; a < (int)n.shape.size(); ++a)
      if (!used[a]) n.mem.push_back(a);
    decided[id] = true;
  };
  for (auto& st : plan.steps) {
    if (st.kind != STEP_CONTRACT) continue;
    arrange(st.x, st.ax, st.y, st.bx);
    arrange(st.y, st.bx, st.x, st.ax);
  }
  // workspace for every intermediate except the final one
  size_t off = 0;
  for (auto& st : plan.steps) {
    if (st.result == plan.final_node) continue;
    Node& n = plan.nodes[st.result];
    int64_t cnt = 1;
    for (int64_t s : n.shape) cnt *= s;
    n.ws_off = off;
    off += align256((size_t)cnt * 4);
  }
  // then the scratch of the split reductions (few long sums)
  plan.scratch_off = off;
  off = align256(off + kReduceScratchBytes);
  // then the k-slice partials: 2^kNetSliceLg results of the largest step
  size_t most = 0;
  for (auto& st : plan.steps) {
    if (st.kind != STEP_CONTRACT) continue;
    size_t cnt = 1;
    for (int64_t s : plan.nodes[st.result].shape) cnt *= (size_t)s;
    most = std::max(most, std::min(cnt << kNetSliceLg, kNetSliceCapFloats));
  }
  plan.slices_off = off;
  plan.slices_floats = most;
  plan.ws_bytes = off + most * 4;
  return TN_OK;
}

// Runs a built plan: validates `out` and the workspace, then one launch
// sequence per step on `stream`.
int32_t run_network(const Plan& plan, int32_t n_nodes, const tn_tensor* nodes, tn_tensor* out, void* workspace,
                    size_t ws_bytes, int32_t prec, void* stream) {
  TN_TRY(check_tensor(out, "out", TN_F32));
  if (plan.ws_bytes > ws_bytes) return fail(TN_ERR_WORKSPACE_TOO_SMALL, "workspace needs %zu bytes", plan.ws_bytes);
  if (plan.ws_bytes > 0 && !workspace) return fail(TN_ERR_INVALID_ARGUMENT, "workspace is NULL");
  const Node& fin = plan.nodes[plan.final_node];
  const int n_out = (int)fin.labels.size();
  if (out->rank != n_out) return fail(TN_ERR_SHAPE_MISMATCH, "out rank %d, network has %d open edges", out->rank, n_out);
  // the final node's axis p holds open label -(q+1): view out with its axes in that order
  tn_tensor fview;
  std::memset(&fview, 0, sizeof(fview));
  fview.data = out->data;
  fview.dtype = TN_F32;
  fview.rank = n_out;
  for (int p = 0; p < n_out; ++p) {
    int q = -fin.labels[p] - 1;
    if (out->shape[q] != fin.shape[p]) return fail(TN_ERR_SHAPE_MISMATCH, "out axis %d has the wrong extent", q);
    fview.shape[p] = fin.shape[p];
    fview.stride[p] = out->stride[q];
  }
  for (int i = 0; i < n_nodes; ++i)
    if (overlaps(*out, nodes[i])) return fail(TN_ERR_ALIASING, "out overlaps node %d", i);
  if (plan.ws_bytes > 0) {
    tn_tensor wsv = make_view(workspace, TN_F32, {(int64_t)(plan.ws_bytes / 4)});
    if (overlaps(*out, wsv)) return fail(TN_ERR_ALIASING, "out overlaps the workspace");
  }
  hipStream_t st = static_cast<hipStream_t>(stream);
  void* scratch = static_cast<char*>(workspace) + plan.scratch_off;
  // contractions that fill few compute units may run as k-slices
  SplitKScope slices(plan.slices_floats ? reinterpret_cast<float*>(static_cast<char*>(workspace) + plan.slices_off)
                                        : nullptr,
                     plan.slices_floats, kNetSliceLg);
  auto view_of = [&](int id) -> tn_tensor {
    const Node& n = plan.nodes[id];
    if (id == plan.final_node) return fview;
    if (n.input >= 0) return nodes[n.input];
    tn_tensor v = contiguous_view(static_cast<char*>(workspace) + n.ws_off, TN_F32, (int32_t)n.shape.size(),
                                  n.shape.data());
    const std::vector<int64_t> st = mem_strides(n);
    for (size_t a = 0; a < st.size(); ++a) v.stride[a] = st[a];
    return v;
  };
  for (auto& s : plan.steps) {
    tn_tensor x = view_of(s.x);
    tn_tensor r = view_of(s.result);
    if (s.kind == STEP_TRACE) {
      TN_TRY(tn_trace_edge(&x, s.ax[0], s.ax[1], &r, stream));
    } else if (s.kind == STEP_CONTRACT) {
      tn_tensor y = view_of(s.y);
      TN_TRY(contract_between_impl(&x, &y, (int32_t)s.ax.size(), s.ax.data(), s.bx.data(), &r, scratch,
                                   kReduceScratchBytes, prec, st));
    } else if (s.kind == STEP_OUTER) {
      tn_tensor y = view_of(s.y);
      TN_TRY(contract_between_impl(&x, &y, 0, nullptr, nullptr, &r, nullptr, 0, prec, st));
    } else {
      std::vector<AxisSpec> ra, ka;
      for (int a = 0; a < x.rank; ++a) ra.push_back({x.shape[a], {x.stride[a], 0, r.stride[a]}});
      TN_TRY(reduce_from_axes(static_cast<const float*>(x.data), nullptr, static_cast<float*>(r.data), ra, ka, false,
                              nullptr, 0, st));
    }
  }
  return TN_OK;
}

// ---------------------------------------------------------------------------
// Scratch of tn_contract_network_noalloc: a static device array, one copy per
// GPU, held until the process ends.  Host code never passes the array's name
// to a kernel (on the host it is only a stand-in symbol): each device's
// address is looked up once, with that device current, and kept.  Nothing
// in it needs to start at zero (every byte a call reads was written earlier
// in the same call), and calls that overlap in time on one GPU race on it.
constexpr size_t kNoAllocScratchBytes = size_t(128) << 20;
__device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices];

int32_t noalloc_scratch(void*& out) {
  int dev = 0;
  TN_TRY(hip_check(hipGetDevice(&dev), "get device"));
  if (dev < 0 || dev >= kMaxDevices) return fail(TN_ERR_UNSUPPORTED, "device %d beyond %d", dev, kMaxDevices);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    TN_TRY(hip_check(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "scratch symbol address"));
    if (!p) return fail(TN_ERR_DEVICE, "scratch symbol address is NULL");
    g_scratch_ptr[dev] = p;
  }
  out = g_scratch_ptr[dev];
  return TN_OK;
}

}  // namespace

}  // namespace tn

using namespace tn;

extern "C" {

int32_t tn_contract_network_workspace(int32_t n_nodes, const tn_tensor* nodes, const int32_t* labels,
                                      const int32_t* offsets, int32_t n_order, const int32_t* order, size_t* bytes) {
  if (!bytes) return fail(TN_ERR_INVALID_ARGUMENT, "bytes is NULL");
  Plan plan;
  TN_TRY(build_plan(n_nodes, nodes, labels, offsets, n_order, order, plan));
  *bytes = plan.ws_bytes;
  return TN_OK;
}

int32_t tn_contract_network(int32_t n_nodes, const tn_tensor* nodes, const int32_t* labels, const int32_t* offsets,
                            int32_t n_order, const int32_t* order, tn_tensor* out, void* workspace, size_t ws_bytes,
                            int32_t prec, void* stream) {
  Plan plan;
  TN_TRY(build_plan(n_nodes, nodes, labels, offsets, n_order, order, plan));
  return run_network(plan, n_nodes, nodes, out, workspace, ws_bytes, prec, stream);
}

int32_t tn_contract_network_noalloc(int32_t n_nodes, const tn_tensor* nodes, const int32_t* labels,
                                    const int32_t* offsets, int32_t n_order, const int32_t* order, tn_tensor* out,
                                    int32_t prec, void* stream) {
  Plan plan;
  TN_TRY(build_plan(n_nodes, nodes, labels, offsets, n_order, order, plan));
  if (plan.ws_bytes > kNoAllocScratchBytes && plan.slices_off <= kNoAllocScratchBytes) {
    // no room for the k-slice partials: every step runs whole
    plan.slices_floats = 0;
    plan.ws_bytes = plan.slices_off;
  }
  if (plan.ws_bytes > kNoAllocScratchBytes)
    return fail(TN_ERR_UNSUPPORTED,
                "network needs %zu bytes of scratch; the library's static scratch holds %zu (use "
                "tn_contract_network with a caller workspace)",
                plan.ws_bytes, (size_t)kNoAllocScratchBytes);
  void* ws = nullptr;
  if (plan.ws_bytes > 0) TN_TRY(noalloc_scratch(ws));
  // the tile tuner never times candidates here (timing creates HIP events)
  NoTimingScope no_timing;
  return run_network(plan, n_nodes, nodes, out, ws, kNoAllocScratchBytes, prec, stream);
}

}  // extern "C"
