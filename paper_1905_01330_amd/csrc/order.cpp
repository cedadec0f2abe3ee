// Contraction order search for ncon networks (host only).  The cost of a
// pairwise contraction is its flop count, 2 x the product of the extents of
// every label on the two nodes (contracted labels once): the product
// C = sum_k A B over all shared labels, as the network driver contracts it.
// Labels traced on one node are contracted first (they shrink that node).
//   greedy : repeatedly contract the connected pair of nodes that is best by
//            one criterion (fewest flops; largest shrink of the network,
//            i.e. result size minus operand sizes; smallest result), one
//            pass per criterion, keeping the pass with the fewest total flops;
//   optimal: exact minimum total flops over all pairwise contraction trees
//            (dynamic programming over subsets of each connected component,
//            at most 12 nodes per component), merging only node sets that
//            share a label, as the driver does, and whose result keeps at
//            most TN_MAX_RANK axes.
// The result is a label order for tn_contract_network: per merge, one label
// shared by the two sides (the driver contracts the others with it).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <vector>

#include "internal.h"

namespace tn {

namespace {

struct OrderNet {
  std::vector<std::vector<int32_t>> labels;   // per node, trace labels removed
  std::map<int32_t, int64_t> dim;              // label -> extent
  std::vector<int32_t> traces;                 // trace labels, in node order
};

int32_t order_setup(int32_t n_nodes, const tn_tensor* nodes, const int32_t* labels, const int32_t* offsets,
                    OrderNet& net) {
  if (n_nodes < 1 || !nodes || !labels || !offsets) return fail(TN_ERR_INVALID_ARGUMENT, "empty network description");
  if (offsets[0] != 0) return fail(TN_ERR_INVALID_ARGUMENT, "offsets[0] must be 0");
  std::map<int32_t, int> count;
  for (int i = 0; i < n_nodes; ++i) {
    if (offsets[i + 1] - offsets[i] != nodes[i].rank)
      return fail(TN_ERR_INVALID_ARGUMENT, "node %d: %d labels for rank %d", i, offsets[i + 1] - offsets[i], nodes[i].rank);
    std::vector<int32_t> ls;
    for (int a = 0; a < nodes[i].rank; ++a) {
      const int32_t l = labels[offsets[i] + a];
      auto it = net.dim.find(l);
      if (it != net.dim.end() && it->second != nodes[i].shape[a])
        return fail(TN_ERR_SHAPE_MISMATCH, "label %d joins axes of different extent", l);
      net.dim[l] = nodes[i].shape[a];
      ++count[l];
      ls.push_back(l);
    }
    // labels appearing twice on this node are traces
    std::vector<int32_t> kept;
    for (int32_t l : ls) {
      if (l >= 0 && std::count(ls.begin(), ls.end(), l) == 2) {
        if (std::find(net.traces.begin(), net.traces.end(), l) == net.traces.end()) net.traces.push_back(l);
      } else {
        kept.push_back(l);
      }
    }
    net.labels.push_back(kept);
  }
  for (auto& kv : count) {
    if (kv.first >= 0 && kv.second != 2) return fail(TN_ERR_INVALID_ARGUMENT, "label %d appears %d times", kv.first, kv.second);
    if (kv.first < 0 && kv.second != 1) return fail(TN_ERR_INVALID_ARGUMENT, "open label %d repeated", kv.first);
  }
  return TN_OK;
}

// labels of the merge of two label sets: the symmetric difference
std::vector<int32_t> merged(const std::vector<int32_t>& a, const std::vector<int32_t>& b) {
  std::vector<int32_t> r;
  for (int32_t l : a)
    if (std::find(b.begin(), b.end(), l) == b.end()) r.push_back(l);
  for (int32_t l : b)
    if (std::find(a.begin(), a.end(), l) == a.end()) r.push_back(l);
  return r;
}

int32_t shared_label(const std::vector<int32_t>& a, const std::vector<int32_t>& b) {
  for (int32_t l : a)
    if (l >= 0 && std::find(b.begin(), b.end(), l) != b.end()) return l;
  return INT32_MIN;
}

double pair_flops(const OrderNet& net, const std::vector<int32_t>& a, const std::vector<int32_t>& b) {
  double f = 2.0;
  for (int32_t l : a) f *= (double)net.dim.at(l);
  for (int32_t l : b)
    if (std::find(a.begin(), a.end(), l) == a.end()) f *= (double)net.dim.at(l);
  return f;
}

double size_of(const OrderNet& net, const std::vector<int32_t>& ls) {
  double s = 1.0;
  for (int32_t l : ls) s *= (double)net.dim.at(l);
  return s;
}

// One greedy pass.  criterion 0: the pair with the fewest flops; 1: the pair
// whose result shrinks the network most (result size minus the two
// operands' sizes); 2: the pair with the smallest result.  Ties: fewer
// flops, then the lower node indices.  strict: pairs whose result has more
// axes than a tensor descriptor holds are never taken, and the pass fails
// (returns false) when only such pairs are left; otherwise they are taken
// only when no other pair joins.  seed != 0: pick at random (a fixed
// linear congruential sequence) among the `pool` best pairs.
bool greedy_pass(const OrderNet& net, int criterion, bool strict, uint32_t seed, int pool, std::vector<int32_t>& order,
                 double& flops) {
  std::vector<std::vector<int32_t>> alive = net.labels;
  std::vector<bool> gone(alive.size(), false);
  uint32_t rnd = seed;
  struct Cand {
    double key, f;
    bool over;
    int i, j;
  };
  for (;;) {
    std::vector<Cand> best;   // up to `pool`, best first
    bool any_pair = false;
    for (size_t i = 0; i < alive.size(); ++i) {
      if (gone[i]) continue;
      for (size_t j = i + 1; j < alive.size(); ++j) {
        if (gone[j] || shared_label(alive[i], alive[j]) == INT32_MIN) continue;
        any_pair = true;
        const std::vector<int32_t> m = merged(alive[i], alive[j]);
        const bool over = (int)m.size() > TN_MAX_RANK;
        if (over && strict) continue;
        const double f = pair_flops(net, alive[i], alive[j]);
        const double sz = size_of(net, m);
        const double key = criterion == 0 ? f
                         : criterion == 1 ? sz - size_of(net, alive[i]) - size_of(net, alive[j])
                                          : sz;
        const Cand c{key, f, over, (int)i, (int)j};
        auto better = [](const Cand& x, const Cand& y) {
          if (x.over != y.over) return !x.over;
          return x.key < y.key || (x.key == y.key && x.f < y.f);
        };
        size_t pos = best.size();
        while (pos > 0 && better(c, best[pos - 1])) --pos;
        if ((int)pos < pool) {
          best.insert(best.begin() + pos, c);
          if ((int)best.size() > pool) best.pop_back();
        }
      }
    }
    if (best.empty()) return !any_pair;   // done, or only over-rank pairs left (strict)
    size_t pick = 0;
    if (seed) {
      rnd = rnd * 1664525u + 1013904223u;
      pick = (rnd >> 16) % best.size();
    }
    const Cand& c = best[pick];
    order.push_back(shared_label(alive[c.i], alive[c.j]));
    flops += c.f;
    alive[c.i] = merged(alive[c.i], alive[c.j]);
    gone[c.j] = true;
  }
}

// The cheapest (total flops) order among: the three strict passes; if none
// completes, 256 seeded random strict passes (the three criteria in turn,
// picking among the best 3 to 5 pairs); if none completes either, the three
// permissive passes (the driver then rejects the over-rank step).
void greedy(const OrderNet& net, std::vector<int32_t>& order, double& flops) {
  std::vector<int32_t> best;
  double best_f = INFINITY;
  auto consider = [&](int c, bool strict, uint32_t seed, int pool) {
    std::vector<int32_t> o;
    double f = 0.0;
    if (greedy_pass(net, c, strict, seed, pool, o, f) && f < best_f) {
      best = o;
      best_f = f;
    }
  };
  for (int c = 0; c < 3; ++c) consider(c, true, 0, 1);
  for (uint32_t t = 1; best_f == INFINITY && t <= 256; ++t)
    consider((int)(t % 3), true, 0x9e3779b9u * t, 3 + (int)(t % 3));
  for (int c = 0; best_f == INFINITY && c < 3; ++c) consider(c, false, 0, 1);
  order.insert(order.end(), best.begin(), best.end());
  flops += best_f;
}

constexpr int kMaxOptimal = 12;

// exact minimum over contraction trees of one connected component
int32_t optimal_component(const OrderNet& net, const std::vector<int>& comp, std::vector<int32_t>& order,
                          double& flops) {
  const int n = (int)comp.size();
  const uint32_t full = (1u << n) - 1;
  std::vector<std::vector<int32_t>> lab(full + 1);
  std::vector<double> cost(full + 1, INFINITY);
  std::vector<uint32_t> split(full + 1, 0);
  for (int i = 0; i < n; ++i) {
    lab[1u << i] = net.labels[comp[i]];
    cost[1u << i] = 0.0;
  }
  for (uint32_t s = 1; s <= full; ++s) {
    if ((s & (s - 1)) == 0) continue;
    // labels of s: those of any split (the symmetric difference is associative)
    const uint32_t low = s & (~s + 1);
    lab[s] = merged(lab[low], lab[s ^ low]);
    // every split s = a + (s - a) with a holding the lowest node (each pair once)
    for (uint32_t a = (s - 1) & s; a > 0; a = (a - 1) & s) {
      if (!(a & low)) continue;
      const uint32_t b = s ^ a;
      if (cost[a] == INFINITY || cost[b] == INFINITY) continue;
      if (shared_label(lab[a], lab[b]) == INT32_MIN) continue;
      // the merge's result must fit a tensor descriptor (the whole set's labels)
      if ((int)lab[s].size() > TN_MAX_RANK) continue;
      const double c = cost[a] + cost[b] + pair_flops(net, lab[a], lab[b]);
      if (c < cost[s]) {
        cost[s] = c;
        split[s] = a;
      }
    }
  }
  if (n > 1 && cost[full] == INFINITY)
    return fail(TN_ERR_UNSUPPORTED, "no contraction order keeps every intermediate within rank %d", TN_MAX_RANK);
  flops += cost[full];
  // post-order: contract both sides, then the merge
  std::vector<std::pair<uint32_t, bool>> stack = {{full, false}};
  while (!stack.empty()) {
    auto [s, expanded] = stack.back();
    stack.pop_back();
    if ((s & (s - 1)) == 0) continue;
    const uint32_t a = split[s], b = s ^ a;
    if (expanded) {
      order.push_back(shared_label(lab[a], lab[b]));
    } else {
      stack.push_back({s, true});
      stack.push_back({b, false});
      stack.push_back({a, false});
    }
  }
  return TN_OK;
}

}  // namespace

}  // namespace tn

using namespace tn;

extern "C" {

int32_t tn_network_order(int32_t n_nodes, const tn_tensor* nodes, const int32_t* labels, const int32_t* offsets,
                         int32_t method, int32_t* order, int32_t* n_order, double* flops) {
  if (!order || !n_order || !flops) return fail(TN_ERR_INVALID_ARGUMENT, "order, n_order or flops is NULL");
  if (method != TN_ORDER_GREEDY && method != TN_ORDER_OPTIMAL) return fail(TN_ERR_INVALID_ARGUMENT, "unknown method %d", method);
  OrderNet net;
  TN_TRY(order_setup(n_nodes, nodes, labels, offsets, net));
  std::vector<int32_t> seq = net.traces;
  double f = 0.0;
  if (method == TN_ORDER_GREEDY) {
    greedy(net, seq, f);
  } else {
    // connected components of the nodes (after the traces)
    std::vector<int> comp_of(net.labels.size(), -1);
    int n_comp = 0;
    for (size_t i = 0; i < net.labels.size(); ++i) {
      if (comp_of[i] >= 0) continue;
      std::vector<int> stack = {(int)i};
      comp_of[i] = n_comp;
      while (!stack.empty()) {
        const int u = stack.back();
        stack.pop_back();
        for (size_t v = 0; v < net.labels.size(); ++v)
          if (comp_of[v] < 0 && shared_label(net.labels[u], net.labels[v]) != INT32_MIN) {
            comp_of[v] = n_comp;
            stack.push_back((int)v);
          }
      }
      ++n_comp;
    }
    for (int c = 0; c < n_comp; ++c) {
      std::vector<int> comp;
      for (size_t i = 0; i < net.labels.size(); ++i)
        if (comp_of[i] == c) comp.push_back((int)i);
      if ((int)comp.size() > kMaxOptimal)
        return fail(TN_ERR_UNSUPPORTED, "optimal order: a component has %zu nodes (at most %d)", comp.size(), kMaxOptimal);
      TN_TRY(optimal_component(net, comp, seq, f));
    }
  }
  // the driver contracts every shared label with the first one: list each
  // connected label once, the first of each merge in merge order, then any
  // label not yet listed (those it contracts alongside)
  std::vector<int32_t> all;
  for (auto& kv : net.dim)
    if (kv.first >= 0) all.push_back(kv.first);
  for (int32_t l : all)
    if (std::find(seq.begin(), seq.end(), l) == seq.end()) seq.push_back(l);
  for (size_t i = 0; i < seq.size(); ++i) order[i] = seq[i];
  *n_order = (int32_t)seq.size();
  *flops = f;
  return TN_OK;
}

}  // extern "C"
