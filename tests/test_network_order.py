"""Contraction order search (host only: reads shapes, no GPU).

Pins: the matrix-chain case worked by hand; the dynamic program's optimum
against an exhaustive search over all pairwise contraction sequences on
small random networks; the reported flops against a simulation of the
network driver following the returned label order; greedy never below the
optimum."""
import functools
import itertools
import random

import pytest
import torch

import paper_1905_01330_amd as tn


def shapes_of(labels, dims):
    return [torch.empty([dims[l] for l in ls]) for ls in labels]


def simulate(labels, dims, order):
    """flops of the driver following `order`: a label joining two nodes
    contracts every label they share (2 x product of all their extents)."""
    nodes = [list(ls) for ls in labels]
    # traces first: labels twice on one node
    for n in nodes:
        for l in set(n):
            if l >= 0 and n.count(l) == 2:
                while l in n:
                    n.remove(l)
    flops = 0.0
    done = set()
    for l in order:
        if l in done:
            continue
        hold = [i for i, n in enumerate(nodes) if n is not None and l in n]
        if len(hold) != 2:
            done.add(l)
            continue
        a, b = nodes[hold[0]], nodes[hold[1]]
        union = set(a) | set(b)
        f = 2.0
        for x in union:
            f *= dims[x]
        flops += f
        shared = set(a) & set(b)
        done |= {x for x in shared if x >= 0}
        nodes[hold[0]] = [x for x in a if x not in shared] + [x for x in b if x not in shared]
        nodes[hold[1]] = None
    return flops


def brute_force(labels, dims):
    """minimum total flops over every sequence of pairwise merges of nodes
    that share a label (exhaustive, memoised on the multiset of nodes)."""
    @functools.lru_cache(maxsize=None)
    def best(state):
        nodes = [set(n) for n in state]
        if len(nodes) == 1:
            return 0.0
        out = float("inf")
        for i, j in itertools.combinations(range(len(nodes)), 2):
            sh = {x for x in nodes[i] & nodes[j] if x >= 0}
            if not sh:
                continue
            f = 2.0
            for x in nodes[i] | nodes[j]:
                f *= dims[x]
            rest = [frozenset(n) for k, n in enumerate(nodes) if k not in (i, j)]
            rest.append(frozenset(nodes[i] ^ nodes[j]))
            out = min(out, f + best(tuple(sorted(rest, key=sorted))))
        return out
    return best(tuple(sorted((frozenset(ls) for ls in labels), key=sorted)))


def test_matrix_chain_by_hand():
    # A[10,100] B[100,5] C[5,50]: (AB)C = 2*10*100*5 + 2*10*5*50 = 15000 flops
    labels = [[-1, 0], [0, 1], [1, -2]]
    dims = {-1: 10, 0: 100, 1: 5, -2: 50}
    for method in ("greedy", "optimal"):
        order, flops = tn.network_order(shapes_of(labels, dims), labels, method)
        assert flops == 15000.0
        assert order[0] == 0
        assert simulate(labels, dims, order) == flops


def random_network(rng, n_nodes, n_open):
    """a connected random graph: a spanning tree plus extra edges"""
    edges = [(rng.randrange(i), i) for i in range(1, n_nodes)]
    for _ in range(rng.randrange(0, n_nodes)):
        i, j = rng.sample(range(n_nodes), 2)
        edges.append((i, j))
    labels = [[] for _ in range(n_nodes)]
    dims = {}
    for lab, (i, j) in enumerate(edges):
        labels[i].append(lab)
        labels[j].append(lab)
        dims[lab] = rng.randint(2, 7)
    for q in range(n_open):
        labels[rng.randrange(n_nodes)].append(-(q + 1))
        dims[-(q + 1)] = rng.randint(2, 7)
    return labels, dims


@pytest.mark.parametrize("seed", range(12))
def test_optimal_matches_exhaustive_search(seed):
    rng = random.Random(seed)
    labels, dims = random_network(rng, rng.randint(3, 6), rng.randint(0, 3))
    ts = shapes_of(labels, dims)
    order_o, flops_o = tn.network_order(ts, labels, "optimal")
    assert abs(flops_o - brute_force(labels, dims)) <= 1e-9 * flops_o
    assert simulate(labels, dims, order_o) == flops_o
    order_g, flops_g = tn.network_order(ts, labels, "greedy")
    assert simulate(labels, dims, order_g) == flops_g
    assert flops_g >= flops_o
    assert sorted(order_o) == sorted(order_g) == sorted(l for l in dims if l >= 0)


def test_traces_first_and_disconnected_parts():
    # node 0 carries a trace (label 5); nodes {0, 1} and {2, 3} are not connected
    labels = [[5, 0, 5, -1], [0, -2], [1, -3], [1, -4]]
    dims = {5: 3, 0: 4, -1: 2, -2: 6, 1: 5, -3: 2, -4: 3}
    for method in ("greedy", "optimal"):
        order, flops = tn.network_order(shapes_of(labels, dims), labels, method)
        assert order[0] == 5
        assert sorted(order) == [0, 1, 5]
        assert flops == 2.0 * 4 * 2 * 6 + 2.0 * 5 * 2 * 3


def test_order_errors():
    labels = [[0, 1], [1, 2], [2, 0]]
    dims = {0: 2, 1: 3, 2: 4}
    ts = shapes_of(labels, dims)
    with pytest.raises(tn.TNError):
        tn.network_order(ts, [[0, 1], [1, 2], [2, 3]], "optimal")      # label 0 and 3 once
    with pytest.raises(tn.TNError):
        tn.network_order([torch.empty(2, 3), torch.empty(4, 4), torch.empty(4, 2)], labels)   # extents differ
    # a ring of 13 nodes exceeds the exact search, greedy still answers
    ring = [[i, (i + 1) % 13] for i in range(13)]
    ts = [torch.empty(2, 2) for _ in range(13)]
    with pytest.raises(tn.TNError):
        tn.network_order(ts, ring, "optimal")
    order, flops = tn.network_order(ts, ring, "greedy")
    assert sorted(order) == list(range(13)) and flops > 0


@pytest.mark.parametrize("ops", [(), (5,), (7, 8), (0, 15)])
def test_greedy_orders_of_mera_networks_fit_the_descriptor_rank(ops):
    """The 16-site binary MERA's <psi|O|psi> networks have pairwise orders
    whose intermediates keep at most 8 axes; the search must find one (the
    driver's planning, host only, accepts it)."""
    import ctypes as C

    import torch

    import paper_1905_01330_amd as tn
    from paper_1905_01330_amd import _lib as L
    from paper_1905_01330_amd import networks

    shapes, labels, _ = networks.expectation(16, 2, 8, ops, True)
    ts = [torch.empty(s) for s in shapes]
    order, flops = tn.network_order(ts, labels, "greedy")
    flat, offs = [], [0]
    for lab in labels:
        flat.extend(lab)
        offs.append(len(flat))
    nb = C.c_size_t(0)
    assert L.lib().tn_contract_network_workspace(len(ts), L.tensor_array(ts), L.int_array(flat), L.int_array(offs),
                                                 len(order), L.int_array(order), C.byref(nb)) == 0
    assert flops < 1e9
