"""Pins of the oracle's contraction primitives against brute force and the paper's examples."""
import itertools
import json
import math
import os

import numpy as np
import pytest

import oracle
from helpers import brute_network, brute_tensordot

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_examples.json")))


def _random_pair_case(rng):
    ra = int(rng.integers(0, 5))
    rb = int(rng.integers(0, 5))
    npairs = int(rng.integers(0, min(ra, rb) + 1))
    pa = list(rng.permutation(ra)[:npairs])
    pb = list(rng.permutation(rb)[:npairs])
    sa = [int(rng.integers(1, 4)) for _ in range(ra)]
    sb = [int(rng.integers(1, 4)) for _ in range(rb)]
    for i, j in zip(pa, pb):
        sb[j] = sa[i]
    return rng.standard_normal(sa), rng.standard_normal(sb), pa, pb


@pytest.mark.parametrize("seed", range(40))
def test_tensordot_matches_brute_force(seed):
    rng = np.random.default_rng(1000 + seed)
    a, b, pa, pb = _random_pair_case(rng)
    got = oracle.tensordot(a, b, pa, pb)
    ref = brute_tensordot(a, b, pa, pb)
    assert got.shape == ref.shape
    np.testing.assert_allclose(got, ref, rtol=1e-13, atol=1e-13)


def test_tensordot_special_cases_reduce_to_textbook_ops():
    # Fig. 2: vector.vector, matrix.vector, matrix.matrix, trace
    rng = np.random.default_rng(7)
    v, w = rng.standard_normal(5), rng.standard_normal(5)
    m, n = rng.standard_normal((4, 5)), rng.standard_normal((5, 3))
    assert math.isclose(float(oracle.tensordot(v, w, [0], [0])), sum(x * y for x, y in zip(v, w)), rel_tol=1e-14)
    mv = [sum(m[i, j] * w[j] for j in range(5)) for i in range(4)]
    np.testing.assert_allclose(oracle.tensordot(m, w, [1], [0]), mv, rtol=1e-14)
    mm = [[sum(m[i, j] * n[j, k] for j in range(5)) for k in range(3)] for i in range(4)]
    np.testing.assert_allclose(oracle.tensordot(m, n, [1], [0]), mm, rtol=1e-13)
    sq = rng.standard_normal((6, 6))
    assert math.isclose(float(oracle.trace_edge(sq, 0, 1)), sum(sq[i, i] for i in range(6)), rel_tol=1e-14)


def test_tensordot_invariant_under_operand_transposition():
    rng = np.random.default_rng(3)
    a = rng.standard_normal((3, 4, 5))
    b = rng.standard_normal((5, 2, 4))
    ref = oracle.tensordot(a, b, [1, 2], [2, 0])
    at = np.transpose(a, (2, 0, 1))   # axes (5,3,4): contracted axes now 2 and 0
    got = oracle.tensordot(at, b, [2, 0], [2, 0])
    np.testing.assert_allclose(got, ref, rtol=1e-13)


def test_golden_ones_dot():
    g = GOLDEN["ones_dot"]
    c = oracle.contract_network([np.array(g["a"]), np.array(g["b"])], [[0], [0]])
    assert float(c) == g["value"]
    assert float(oracle.contract_between(np.array(g["a"]), np.array(g["b"]), [(0, 0)])) == g["value"]


def test_golden_outer_shape_and_values():
    g = GOLDEN["outer_shape"]
    rng = np.random.default_rng(5)
    a = rng.standard_normal(g["shape_a"])
    b = rng.standard_normal(g["shape_b"])
    c = oracle.outer_product(a, b)
    assert list(c.shape) == g["shape_out"]
    for idx in itertools.product(*[range(s) for s in g["shape_out"]]):
        assert c[idx] == a[idx[:2]] * b[idx[2:]]


def test_golden_ncon_matmul():
    g = GOLDEN["ncon_matmul"]
    rng = np.random.default_rng(11)
    a = rng.standard_normal(g["shape_a"])
    b = rng.standard_normal(g["shape_b"])
    c = oracle.contract_network([a, b], g["labels"])
    mm = np.array([[sum(a[i, j] * b[j, k] for j in range(2)) for k in range(2)] for i in range(2)])
    assert np.linalg.norm(c - mm) <= 1e-15 + g["difference_norm"]


def test_trace_matches_loops():
    rng = np.random.default_rng(9)
    a = rng.standard_normal((3, 4, 2, 4))
    got = oracle.trace_edge(a, 1, 3)
    ref = np.zeros((3, 2))
    for i in range(3):
        for j in range(2):
            ref[i, j] = sum(a[i, q, j, q] for q in range(4))
    np.testing.assert_allclose(got, ref, rtol=1e-14)
    assert float(oracle.trace_edge(np.eye(7), 0, 1)) == 7.0


def test_flatten_example_eye():
    # III.B "Edge Flattening": two eye(2) nodes joined on both edges; the
    # flattened single edge has dimension 4 and the contraction is Tr(I I^T) = 2.
    c = oracle.contract_network([np.eye(2), np.eye(2)], [[0, 1], [0, 1]])
    assert float(c) == 2.0


def test_parallel_edges_one_at_a_time_equal_flattening():
    # III.B: contracting one of two parallel edges leaves a trace edge; the value is the same.
    rng = np.random.default_rng(21)
    a = rng.standard_normal((3, 4, 5))
    b = rng.standard_normal((4, 6, 3))
    flat = oracle.contract_between(a, b, [(0, 2), (1, 0)])        # [5, 6]
    step = oracle.tensordot(a, b, [0], [2])                         # [4, 5, 4, 6]
    step = oracle.trace_edge(step, 0, 2)                            # [5, 6]
    np.testing.assert_allclose(step, flat, rtol=1e-13)


def test_hadamard_chain():
    # III.B "Connecting Dangling Edges": five Hadamards applied to |0>; since H^2 = I
    # the result is H|0> = (1, 1)/sqrt(2).
    h = np.array([[1.0, 1.0], [1.0, -1.0]]) / np.sqrt(2.0)
    tensors = [np.array([1.0, 0.0])] + [h] * 5
    labels = [[0]] + [[i + 1, i] for i in range(4)] + [[-1, 4]]
    out = oracle.contract_network(tensors, labels)
    np.testing.assert_allclose(out, [1 / np.sqrt(2), 1 / np.sqrt(2)], rtol=1e-14)


def _small_network(rng):
    # four nodes with a trace edge, a double edge and three open legs
    t0 = rng.standard_normal((2, 3, 3, 2))   # labels 0, 9, 9(trace), 1
    t1 = rng.standard_normal((2, 2, 3))      # labels 0, 2, -2
    t2 = rng.standard_normal((2, 2, 2, 2))   # labels 1, 2, 3, -1
    t3 = rng.standard_normal((2, 2))         # labels 3, -3
    return [t0, t1, t2, t3], [[0, 9, 9, 1], [0, 2, -2], [1, 2, 3, -1], [3, -3]]


def test_network_matches_brute_force():
    rng = np.random.default_rng(31)
    ts, ls = _small_network(rng)
    got = oracle.contract_network(ts, ls)
    ref = brute_network(ts, ls)
    assert got.shape == (2, 3, 2)
    np.testing.assert_allclose(got, ref, rtol=1e-12, atol=1e-13)


def test_network_order_invariance():
    rng = np.random.default_rng(32)
    ts, ls = _small_network(rng)
    ref = oracle.contract_network(ts, ls)
    for order in itertools.permutations([0, 1, 2, 3, 9]):
        got = oracle.contract_network(ts, ls, list(order))
        np.testing.assert_allclose(got, ref, rtol=1e-12, atol=1e-14)


def test_network_disconnected_is_outer_product():
    rng = np.random.default_rng(33)
    a, b = rng.standard_normal((2, 3)), rng.standard_normal(4)
    got = oracle.contract_network([a, b], [[-3, -1], [-2]])
    ref = np.transpose(oracle.outer_product(a, b), (1, 2, 0))
    np.testing.assert_array_equal(got, ref)


def test_feature_map_unit_norm_and_one_hot():
    # IV.A: Phi(p) = (cos pi p/2, sin pi p/2); p in {0, 1} is the one-hot encoding.
    p = np.linspace(0, 1, 101)
    f = oracle.feature_map(p)
    np.testing.assert_allclose(np.sum(f * f, axis=1), 1.0, rtol=1e-15)
    np.testing.assert_allclose(oracle.feature_map(0.0), [1.0, 0.0], atol=1e-16)
    np.testing.assert_allclose(oracle.feature_map(1.0), [0.0, 1.0], atol=1e-16)


def test_rejects_bad_input():
    with pytest.raises(ValueError):
        oracle.tensordot(np.ones((2, 3)), np.ones((4,)), [1], [0])
    with pytest.raises(ValueError):
        oracle.contract_network([np.ones(2), np.ones(2)], [[0], [1]])
