"""Pins of the oracle's network contraction on tree-like states (section II,
TTN and MERA): the dense state vector is an independent route to local
expectation values, and networks of isometries have norm equal to the
root's (exactly 1 for a unit root)."""
import numpy as np
import pytest

import oracle
from helpers import greedy_order, random_orthogonal
from paper_1905_01330_amd import networks

Z = np.diag([1.0, -1.0])
X = np.array([[0.0, 1.0], [1.0, 0.0]])


def random_tensors(net, seed):
    rng = np.random.default_rng(seed)
    return [rng.standard_normal(s) / np.sqrt(np.prod(s[:2])) for s in net.shapes]


def isometric_tensors(net, seed):
    """w: orthonormal columns over (lower1, lower2); u: orthogonal over
    (lower1 lower2) -> (upper1 upper2); root with unit norm."""
    rng = np.random.default_rng(seed)
    out = []
    for kind, s in zip(net.kinds, net.shapes):
        if kind == "root":
            r = rng.standard_normal(s)
            out.append(r / np.linalg.norm(r))
        elif kind == "w":
            q = random_orthogonal(s[0] * s[1], rng)[:, :s[2]]
            out.append(q.reshape(s))
        else:
            out.append(random_orthogonal(s[0] * s[1], rng).reshape(s))
    return out


def dense_state(n, d, chi, mera, tensors):
    net, _ = networks.tree_state(n, d, chi, mera)
    return oracle.contract_network(tensors, net.labels, greedy_order(net.shapes, net.labels)).reshape(-1)


def op_dense(n, ops):
    """Dense product operator (site 0 most significant, as the output axes -1, -2, ...)."""
    m = np.ones((1, 1))
    for i in range(n):
        m = np.kron(m, ops.get(i, np.eye(2)))
    return m


@pytest.mark.parametrize("mera", [False, True])
def test_isometric_networks_have_unit_norm(mera):
    n = 16
    net, _ = networks.tree_state(n, 2, 4, mera)
    t = isometric_tensors(net, 3)
    shapes, labels, src = networks.expectation(n, 2, 4, (), mera)
    val = oracle.contract_network([t[i] for i in src], labels, greedy_order(shapes, labels))
    assert abs(float(val) - 1.0) < 1e-12


@pytest.mark.parametrize("mera", [False, True])
def test_expectations_match_the_dense_state(mera):
    n, d, chi = 8, 2, 4
    net, _ = networks.tree_state(n, d, chi, mera)
    t = random_tensors(net, 5)
    psi = dense_state(n, d, chi, mera, t)
    for ops in ({}, {2: Z, 3: Z}, {5: X}, {0: Z, 7: X}):
        shapes, labels, src = networks.expectation(n, d, chi, tuple(sorted(ops)), mera)
        nodes = []
        it = iter(sorted(ops))
        for i in src:
            nodes.append(t[i] if i >= 0 else ops[next(it)])
        val = float(oracle.contract_network(nodes, labels, greedy_order(shapes, labels)))
        want = float(psi @ op_dense(n, ops) @ psi)
        assert abs(val - want) <= 1e-12 * float(psi @ psi), (ops, val, want)


def test_structure_counts():
    net, _ = networks.tree_state(16, 2, 8, False)
    assert len(net.shapes) == 15 and net.kinds.count("root") == 1
    assert net.shapes[-1] == (8, 8)
    m, _ = networks.tree_state(16, 2, 8, True)
    # disentanglers: 7 at the first level, 3 at the second, 1 at the third
    assert m.kinds.count("u") == 7 + 3 + 1 and m.kinds.count("w") == 8 + 4 + 2
