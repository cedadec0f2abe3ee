"""Pins of the node-splitting oracle (section III.B "Node Splitting",
Appendix A "Saving Memory"): the paper's shapes, a spectrum known by
construction, the truncation rule against brute force, Eckart-Young, and
the properties every SVD has."""
import json
import os

import numpy as np
import pytest

import oracle
from helpers import random_orthogonal

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_examples.json")))


def known_spectrum(m, n, s, seed):
    """A = Q1[:, :r] diag(s) Q2[:, :r]^T with random orthogonal Q1, Q2: its
    singular values are s (any order) by construction."""
    rng = np.random.default_rng(seed)
    r = len(s)
    q1 = random_orthogonal(m, rng)[:, :r]
    q2 = random_orthogonal(n, rng)[:, :r]
    return (q1 * np.asarray(s)[None, :]) @ q2.T


def test_golden_split_shapes():
    g = GOLDEN["split_shapes"]
    a = np.random.default_rng(1).standard_normal(g["shape"])
    left, right, trun = oracle.split_node(a, g["n_left"])
    assert list(left.shape) == g["left_shape"] and list(right.shape) == g["right_shape"]
    assert trun.shape == (0,)
    u, s, vt, trun = oracle.split_node_full_svd(a, g["n_left"])
    assert list(u.shape) == g["left_shape"] and s.shape == (g["new_dim"], g["new_dim"])
    assert list(vt.shape) == g["right_shape"]


def test_golden_truncation_shapes_and_bound():
    g = GOLDEN["split_truncation"]
    # a decaying spectrum, so that the error bound keeps a proper subset
    s = np.exp(-np.arange(1000) / 40.0)
    a = known_spectrum(1000, 1000, s, 7)
    left, right, trun = oracle.split_node(a, 1, max_singular_values=g["max_singular_values"])
    assert list(left.shape) == g["left_shape"] and list(right.shape) == g["right_shape"]
    assert list(trun.shape) == g["trun_err_shape"]
    assert a.size // (left.size + right.size) == g["memory_ratio"]
    left, right, trun = oracle.split_node(a, 1, max_truncation_err=g["max_truncation_err"])
    assert np.sum(trun) <= g["max_truncation_err"]
    # and no more could have been dropped
    k = left.shape[-1]
    assert np.sum(trun) + s[k - 1] > g["max_truncation_err"]


def test_known_spectrum_is_recovered_in_order():
    s = np.array([3.0, 0.25, 7.5, 1.0, 1e-3, 0.5])
    a = known_spectrum(9, 8, s, 3)
    u, sm, vt, trun = oracle.split_node_full_svd(a.reshape(3, 3, 8), 2, max_singular_values=4)
    want = np.sort(s)[::-1]
    np.testing.assert_allclose(np.diag(sm), want[:4], rtol=1e-13)
    # the dropped values come largest first; the two of the 8-wide spectrum that
    # are not in s are exact zeros of this rank-6 matrix
    np.testing.assert_allclose(trun[:2], want[4:], rtol=1e-10)
    assert np.all(np.abs(trun[2:]) < 1e-13)


@pytest.mark.parametrize("seed", range(6))
def test_truncation_rule_against_brute_force(seed):
    """Each limit by enumeration over every rank k = 0..n: the count limit
    keeps min(n, max_sv); the error limit keeps the smallest k whose dropped
    values s[k:] add up to at most the bound; the smaller wins, at least 1."""
    rng = np.random.default_rng(seed)
    s = np.sort(rng.exponential(1.0, 7))[::-1]
    n = len(s)
    for max_sv in (None, 1, 3, 7, 9):
        for err in (None, 0.0, 0.3, 1.0, 2.5, 100.0):
            k_count = n if max_sv is None else min(n, max_sv)
            k_err = n
            if err is not None:
                k_err = min(k for k in range(n + 1) if sum(s[j] for j in range(k, n)) <= err)
            assert oracle.truncation_rank(s, max_sv, err) == max(1, min(k_count, k_err)), (max_sv, err)


@pytest.mark.parametrize("shape,n_left", [((6, 5), 1), ((3, 4, 5), 1), ((3, 4, 5), 2), ((2, 3, 2, 5), 2), ((7, 2, 3), 1)])
def test_factors_reconstruct_and_are_isometries(shape, n_left):
    a = np.random.default_rng(11).standard_normal(shape)
    left, right, _ = oracle.split_node(a, n_left)
    np.testing.assert_allclose(np.tensordot(left, right, 1), a, atol=1e-13)
    u, s, vt, _ = oracle.split_node_full_svd(a, n_left)
    k = s.shape[0]
    um, vm = u.reshape(-1, k), vt.reshape(k, -1)
    np.testing.assert_allclose(um.T @ um, np.eye(k), atol=1e-13)
    np.testing.assert_allclose(vm @ vm.T, np.eye(k), atol=1e-13)
    assert np.all(np.diff(np.diag(s)) <= 0) and np.all(np.diag(s) >= 0)
    # the square roots split evenly: column norms of U sqrt(S) are sqrt(s)
    np.testing.assert_allclose(np.linalg.norm(left.reshape(-1, k), axis=0) ** 2, np.diag(s), rtol=1e-12)
    np.testing.assert_allclose(np.linalg.norm(right.reshape(k, -1), axis=1) ** 2, np.diag(s), rtol=1e-12)


def test_eckart_young_error_of_the_truncated_product():
    """||A - A_k||_F^2 equals the sum of the squared dropped values."""
    a = np.random.default_rng(5).standard_normal((40, 30))
    for k in (1, 5, 17, 30):
        left, right, trun = oracle.split_node(a, 1, max_singular_values=k)
        err2 = np.sum((a - left @ right) ** 2)
        assert abs(err2 - np.sum(trun ** 2)) <= 1e-10 * np.sum(a ** 2)


def test_rank_one_outer_product():
    rng = np.random.default_rng(2)
    x, y = rng.standard_normal(6), rng.standard_normal(9)
    u, s, vt, trun = oracle.split_node_full_svd(np.multiply.outer(x, y), 1)
    assert abs(s[0, 0] - np.linalg.norm(x) * np.linalg.norm(y)) < 1e-13 * s[0, 0]
    assert np.all(np.diag(s)[1:] < 1e-14 * s[0, 0])
    # a zero error bound still drops the exact zeros' neighbours only up to the bound
    _, _, trun = oracle.split_node(np.multiply.outer(x, y), 1, max_truncation_err=1e-10)
    assert len(trun) == 5 and np.sum(trun) <= 1e-10


def test_diagonal_matrix_singular_values_are_sorted_magnitudes():
    d = np.array([-2.0, 0.5, 3.0, -0.25])
    _, s, _, _ = oracle.split_node_full_svd(np.diag(d), 1)
    np.testing.assert_allclose(np.diag(s), np.sort(np.abs(d))[::-1], rtol=1e-15)
