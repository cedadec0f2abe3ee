"""Test-side helpers: brute-force references, dense Hamiltonians and exact MPS builders.

These are independent routes used to pin the oracle: explicit index loops,
Kronecker-product Hamiltonians written from Pauli strings, exact
diagonalisation, and states whose energies are known in closed form.
"""
from __future__ import annotations

import itertools
import math

import numpy as np


# --------------------------------------------------------------------------
# brute force contractions (pure Python loops, tiny sizes only)
# --------------------------------------------------------------------------


def brute_tensordot(a, b, axes_a, axes_b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    free_a = [i for i in range(a.ndim) if i not in axes_a]
    free_b = [j for j in range(b.ndim) if j not in axes_b]
    out_shape = [a.shape[i] for i in free_a] + [b.shape[j] for j in free_b]
    kdims = [a.shape[i] for i in axes_a]
    out = np.zeros(out_shape)
    for oidx in itertools.product(*[range(s) for s in out_shape]):
        ia = [0] * a.ndim
        ib = [0] * b.ndim
        for p, i in enumerate(free_a):
            ia[i] = oidx[p]
        for p, j in enumerate(free_b):
            ib[j] = oidx[len(free_a) + p]
        acc = 0.0
        for kidx in itertools.product(*[range(s) for s in kdims]):
            for p, (i, j) in enumerate(zip(axes_a, axes_b)):
                ia[i] = kidx[p]
                ib[j] = kidx[p]
            acc += a[tuple(ia)] * b[tuple(ib)]
        out[oidx] = acc
    return out


def brute_network(tensors, labels):
    """Full sum over every connected label of the product of all entries (loops)."""
    all_labels = sorted({x for l in labels for x in l})
    dims = {}
    for t, l in zip(tensors, labels):
        for ax, x in enumerate(l):
            dims[x] = t.shape[ax]
    closed = [x for x in all_labels if x >= 0]
    opened = sorted([x for x in all_labels if x < 0], reverse=True)  # -1, -2, ...
    out = np.zeros([dims[x] for x in opened])
    for oidx in itertools.product(*[range(dims[x]) for x in opened]):
        assign = dict(zip(opened, oidx))
        acc = 0.0
        for cidx in itertools.product(*[range(dims[x]) for x in closed]):
            assign.update(zip(closed, cidx))
            prod = 1.0
            for t, l in zip(tensors, labels):
                prod *= t[tuple(assign[x] for x in l)]
            acc += prod
        out[oidx] = acc
    return out


# --------------------------------------------------------------------------
# dense spin-chain Hamiltonians from Pauli strings
# --------------------------------------------------------------------------

PX = np.array([[0, 1], [1, 0]], dtype=complex)
PY = np.array([[0, -1j], [1j, 0]], dtype=complex)
PZ = np.array([[1, 0], [0, -1]], dtype=complex)
I2 = np.eye(2, dtype=complex)


def _site_op(op, i, n):
    m = np.ones((1, 1), dtype=complex)
    for k in range(n):
        m = np.kron(m, op if k == i else I2)
    return m


def dense_tfim(n, J=1.0, g=1.0):
    h = np.zeros((2 ** n, 2 ** n), dtype=complex)
    for i in range(n - 1):
        h -= J * _site_op(PZ, i, n) @ _site_op(PZ, i + 1, n)
    for i in range(n):
        h -= g * _site_op(PX, i, n)
    return h.real


def dense_xxz(n, delta):
    h = np.zeros((2 ** n, 2 ** n), dtype=complex)
    for i in range(n - 1):
        for op, c in ((PX, 1.0), (PY, 1.0), (PZ, delta)):
            h += c * 0.25 * _site_op(op, i, n) @ _site_op(op, i + 1, n)
    assert np.abs(h.imag).max() < 1e-14
    return h.real


def tfim_ground_energy_closed_form(n):
    """Open critical TFIM (J = g = 1): E0 = 1 - 1/sin(pi / (2 (2N + 1)))."""
    return 1.0 - 1.0 / math.sin(math.pi / (2.0 * (2 * n + 1)))


def xx_ground_energy_closed_form(n):
    """XX chain (delta = 0): free fermions with levels cos(pi k/(N+1)); fill the negative ones."""
    lv = [math.cos(math.pi * k / (n + 1)) for k in range(1, n + 1)]
    return sum(x for x in lv if x < 0)


# --------------------------------------------------------------------------
# exact MPS builders
# --------------------------------------------------------------------------


def dense_to_mps(vec, n, d=2):
    """Exact MPS of a dense state by successive SVDs (no truncation)."""
    sites = []
    rest = np.asarray(vec, dtype=np.float64).reshape(1, -1)
    dl = 1
    for k in range(n - 1):
        m = rest.reshape(dl * d, -1)
        u, s, vt = np.linalg.svd(m, full_matrices=False)
        sites.append(u.reshape(dl, d, -1))
        rest = s[:, None] * vt
        dl = u.shape[1]
    sites.append(rest.reshape(dl, d, 1))
    return sites


def random_orthogonal(n, rng):
    q, r = np.linalg.qr(rng.standard_normal((n, n)))
    return q * np.sign(np.diag(r))[None, :]


def product_state_mps(local_vectors, dims, rng, n_gauges=3):
    """Product state written with full-rank dense bond matrices.

    A_k[a, s, b] = v_k[s] M_k[a, b] with M_k = G_k^T E_k G_{k+1}, where E_k
    is the D_k x D_{k+1} identity embedding and G_k are random orthogonal
    matrices (G_0 = G_N = [[1]]; a few distinct ones are cycled along the
    chain).  The bond matrices telescope, M_0 M_1 ... M_{N-1} = [[1]], so the
    state is exactly the product of the local vectors: its norm and energies
    keep their closed forms while every site tensor is dense.
    """
    n = len(local_vectors)
    gauges, mats = {}, {}

    def gauge(k):
        if dims[k] == 1:
            return np.ones((1, 1))
        key = (dims[k], k % n_gauges)
        if key not in gauges:
            gauges[key] = random_orthogonal(dims[k], rng)
        return gauges[key]

    sites = []
    for k in range(n):
        key = (dims[k], dims[k + 1], k % n_gauges if dims[k] > 1 else -1, (k + 1) % n_gauges if dims[k + 1] > 1 else -1)
        if key not in mats:
            mats[key] = gauge(k).T @ np.eye(dims[k], dims[k + 1]) @ gauge(k + 1)
        v = np.asarray(local_vectors[k], dtype=np.float64)
        sites.append(mats[key][:, None, :] * v[None, :, None])
    return sites


def spin_angle_vector(theta):
    """cos(theta/2)|0> + sin(theta/2)|1>: <Z> = cos(theta), <X> = sin(theta)."""
    return np.array([math.cos(theta / 2), math.sin(theta / 2)])


# --------------------------------------------------------------------------
# error measures
# --------------------------------------------------------------------------


def rel_fro(x, ref):
    x = np.asarray(x, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    den = np.linalg.norm(ref.ravel())
    num = np.linalg.norm((x - ref).ravel())
    return num / den if den > 0 else num


def scalar_ms_rel(m, s, m_ref, s_ref):
    """|m e^s / (m_ref e^s_ref) - 1| for (mantissa, log-scale) pairs."""
    return abs(m / m_ref * math.exp(s - s_ref) - 1.0)


# --------------------------------------------------------------------------
# measured-error report (GPU parity runs)
# --------------------------------------------------------------------------


def report(name, **values):
    """Append one JSON line {"case": name, ...} to $TN_PARITY_REPORT, if set.

    GPU parity tests call this with the errors they measured, so a run can
    keep the numbers (including those of precisions that are reported but
    not gated) next to its pass/fail record."""
    import json
    import os

    path = os.environ.get("TN_PARITY_REPORT")
    if not path:
        return
    rec = {"case": name}
    for k, v in values.items():
        rec[k] = float(v) if isinstance(v, (np.floating, float)) else v
    with open(path, "a") as f:
        f.write(json.dumps(rec) + "\n")


def energy_abs_scale(psi, mpo, ls_ref, rs_ref):
    """Sum of |products| of the last contraction on each side (left: L_{N-1}
    with site N-1, right: R_1 with site 0), from the oracle's environments.

    The energy is one number formed by cancelling sums; its rounding error
    is bounded relative to this scale, not to |E|."""
    import oracle

    n = len(psi)
    el = oracle.env_left_step(np.abs(ls_ref[n - 1]), np.abs(psi[n - 1]), np.abs(mpo[n - 1]))[0, 0, 0]
    er = oracle.env_right_step(np.abs(rs_ref[1]), np.abs(psi[0]), np.abs(mpo[0]))[0, 0, 0]
    return float(el), float(er)


# --------------------------------------------------------------------------
# contraction order for the oracle on large networks (test side, independent
# of the library's own search)
# --------------------------------------------------------------------------


def greedy_order(shapes, labels):
    """A label order for oracle.contract_network: repeatedly join the two
    connected nodes whose joint result has the fewest elements (ties: the
    pair found first).  Trace labels come first.  Plain Python over the
    structure only."""
    nodes = [dict(zip(map(int, l), map(int, s))) for s, l in zip(shapes, labels)]
    order = []
    # traces: a label twice on one node
    for i, l in enumerate(labels):
        dup = {x for x in l if list(l).count(x) == 2 and x >= 0}
        order.extend(sorted(dup))
    live = [dict(nd) for nd in nodes]
    alive = list(range(len(live)))
    while True:
        best = None
        for ai in range(len(alive)):
            for bi in range(ai + 1, len(alive)):
                a, b = live[alive[ai]], live[alive[bi]]
                shared = [x for x in a if x in b]
                if not shared:
                    continue
                size = 1
                for x, dx in a.items():
                    if x not in b:
                        size *= dx
                for x, dx in b.items():
                    if x not in a:
                        size *= dx
                if best is None or size < best[0]:
                    best = (size, ai, bi, shared)
        if best is None:
            break
        _, ai, bi, shared = best
        ia, ib = alive[ai], alive[bi]
        order.extend(sorted(shared))
        merged = {x: dx for x, dx in live[ia].items() if x not in live[ib]}
        merged.update({x: dx for x, dx in live[ib].items() if x not in live[ia]})
        live.append(merged)
        alive = [k for k in alive if k not in (ia, ib)] + [len(live) - 1]
    return order
