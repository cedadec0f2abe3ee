"""Oracle: the two-site DMRG update (FP64).

Test infrastructure only (see the package docstring).

Section III.B ("Node Splitting") names DMRG as the algorithm that splits
nodes: the ground state of a chain Hamiltonian is sought as an MPS by
optimising two neighbouring sites at a time.  With the left environment
L[a', u, a] of sites 0..k-1 and the right environment R[b', x, b] of sites
k+2..N-1 (the layouts of the environment sweep), the effective Hamiltonian
on the two-site tensor theta[a, s1, s2, b] is the contraction

  (H_eff theta)[a', t1, t2, b'] =
      sum L[a', u, a] W_k[u, v, t1, s1] W_{k+1}[v, x, t2, s2] R[b', x, b] theta[a, s1, s2, b].

The update replaces theta by the eigenvector of H_eff with the lowest
eigenvalue (numpy's eigh of the dense H_eff is the library step) and splits
it back into two sites with split_node (section III.B), truncated to at
most chi_max singular values: U stays on site k (left-canonical) and S V^T
moves to site k+1 when sweeping to the right; the mirror when sweeping left.
"""
from __future__ import annotations

import numpy as np

from .contract import tensordot
from .mps import env_left_step, env_right_step
from .split import split_node_full_svd


def heff_apply(l, r, w1, w2, theta):
    """H_eff theta, contracted in the order L, W_k, W_{k+1}, R."""
    x1 = tensordot(l, theta, [2], [0])                 # [a', u, s1, s2, b]
    x2 = tensordot(x1, w1, [1, 2], [0, 3])             # [a', s2, b, v, t1]
    x3 = tensordot(x2, w2, [3, 1], [0, 3])             # [a', b, t1, x, t2]
    out = tensordot(x3, r, [1, 3], [2, 1])             # [a', t1, t2, b']
    return out


def heff_dense(l, r, w1, w2):
    """The dense matrix of H_eff on the flattened two-site space (column j = H_eff e_j)."""
    shape = (l.shape[2], w1.shape[3], w2.shape[3], r.shape[2])
    n = int(np.prod(shape))
    h = np.empty((n, n))
    for j in range(n):
        e = np.zeros(n)
        e[j] = 1.0
        h[:, j] = heff_apply(l, r, w1, w2, e.reshape(shape)).ravel()
    return h


def two_site_update(l, r, w1, w2, chi_max=None, direction="right"):
    """Lowest eigenpair of H_eff and the split of its eigenvector.

    Returns (energy, theta, a_left, a_right, trun_err): with direction
    "right", a_left = U (left-canonical) and a_right = S V^T; with "left",
    a_left = U S and a_right = V^T (right-canonical)."""
    shape = (l.shape[2], w1.shape[3], w2.shape[3], r.shape[2])
    h = heff_dense(l, r, w1, w2)
    vals, vecs = np.linalg.eigh(0.5 * (h + h.T))
    theta = vecs[:, 0].reshape(shape)
    u, s, vt, trun = split_node_full_svd(theta, 2, max_singular_values=chi_max)
    if direction == "right":
        return float(vals[0]), theta, u, tensordot(s, vt, [1], [0]), trun
    return float(vals[0]), theta, tensordot(u, s, [2], [0]), vt, trun


def dmrg(mpo, psi0, chi_max, sweeps=2):
    """Two-site DMRG by repeated updates, sweeping right then left.

    psi0 must be right-canonical (sites 1..N-1) so that the right
    environments describe orthonormal bases; returns (energy after each
    update, final sites)."""
    n = len(psi0)
    psi = [np.asarray(x, dtype=np.float64) for x in psi0]
    rs = [None] * (n + 1)
    rs[n] = np.ones((1, 1, 1))
    for k in range(n - 1, 1, -1):
        rs[k] = env_right_step(rs[k + 1], psi[k], mpo[k])
    ls = [None] * (n + 1)
    ls[0] = np.ones((1, 1, 1))
    energies = []
    for _ in range(sweeps):
        for k in range(0, n - 1):                       # left to right
            e, _, a, b, _ = two_site_update(ls[k], rs[k + 2], mpo[k], mpo[k + 1], chi_max, "right")
            psi[k], psi[k + 1] = a, b
            ls[k + 1] = env_left_step(ls[k], psi[k], mpo[k])
            energies.append(e)
        for k in range(n - 2, -1, -1):                  # right to left
            e, _, a, b, _ = two_site_update(ls[k], rs[k + 2], mpo[k], mpo[k + 1], chi_max, "left")
            psi[k], psi[k + 1] = a, b
            rs[k + 1] = env_right_step(rs[k + 2], psi[k + 1], mpo[k + 1])
            energies.append(e)
    return energies, psi
