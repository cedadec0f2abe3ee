"""Oracle: MPS inner products, environment sweeps and canonicalisation (FP64).

Test infrastructure only (see the package docstring).

The MPS is the chain network of Fig. 3a; the inner product of two chains
and the operator expectation are contractions of the kind described in
section III (sums over connected indices), taken site by site from the left
(transfer-matrix order).  Layouts: A_k[D_k, d, D_{k+1}], W_k[w_k, w_{k+1}, t, s],
L_k[bra, mpo, ket].  Real arithmetic: conjugation is the identity.
"""
from __future__ import annotations

import math

import numpy as np

from .contract import tensordot


def mps_inner(psi, phi, rescale=True):
    """<psi|phi> = sum over all physical indices of prod_k psi_k[s_k] * prod_k phi_k[s_k].

    Left-to-right recursion E_0 = [[1]],
      E_{k+1}[b', b] = sum_{a', s} psi_k[a', s, b'] sum_a E_k[a', a] phi_k[a, s, b].
    With rescale, E is divided by max|E| after every site and the logarithm is
    kept in s, so the value is m * exp(s).  Returns (m, s).
    """
    e = np.ones((1, 1))
    logs = 0.0
    for a, b in zip(psi, phi):
        t = tensordot(e, b, [1], [0])                  # [a', s, b]
        e = tensordot(a, t, [0, 1], [0, 1])            # [b', b]
        if rescale:
            mx = float(np.max(np.abs(e)))
            if mx > 0 and np.isfinite(mx):
                e = e / mx
                logs += math.log(mx)
    assert e.shape == (1, 1)
    return float(e[0, 0]), logs


def mps_inner_right(psi, phi):
    """Same value from the right end: F_N = [[1]], F_k = psi_k F_{k+1} phi_k."""
    f = np.ones((1, 1))
    logs = 0.0
    for a, b in zip(reversed(psi), reversed(phi)):
        t = tensordot(b, f, [2], [1])                  # [a, s, b']
        f = tensordot(a, t, [1, 2], [1, 2])            # [a', a]
        mx = float(np.max(np.abs(f)))
        if mx > 0:
            f = f / mx
            logs += math.log(mx)
    return float(f[0, 0]), logs


def mps_inner_value(psi, phi):
    m, s = mps_inner(psi, phi)
    return m * math.exp(s)


def mps_to_dense(mps):
    """Dense 2^N (d^N) state: amplitude(s_1..s_N) = product of the matrices A_k[:, s_k, :].

    Built amplitude by amplitude (vectorised over basis states), an independent
    route from the transfer-matrix sweep.  Basis index is s_1 most significant.
    """
    n = len(mps)
    d = mps[0].shape[1]
    idx = np.arange(d ** n)
    digits = [(idx // d ** (n - 1 - k)) % d for k in range(n)]
    acc = mps[0][0, digits[0], :][:, None, :]          # [S, 1, D1]
    for k in range(1, n):
        mats = np.transpose(mps[k], (1, 0, 2))[digits[k]]   # [S, Dk, Dk+1]
        acc = np.matmul(acc, mats)
    return acc[:, 0, 0]


def mpo_to_dense(mpo):
    """Dense operator (d^N x d^N, row = bra t, column = ket s) from W_k[u, v, t, s]."""
    n = len(mpo)
    d = mpo[0].shape[2]
    dim = d ** n
    idx = np.arange(dim)
    digits = [(idx // d ** (n - 1 - k)) % d for k in range(n)]
    h = np.zeros((dim, dim))
    # amplitude H[t..., s...] = prod_k W_k[:, :, t_k, s_k] (a product of w x w matrices)
    for r in range(dim):
        acc = np.ones((dim, 1, 1))
        for k in range(n):
            m = mpo[k][:, :, digits[k][r], :]           # [u, v, s]
            mats = np.transpose(m, (2, 0, 1))[digits[k]]  # [S, u, v]
            acc = np.matmul(acc, mats)
        h[r, :] = acc[:, 0, 0]
    return h


def left_canonicalize(mps):
    """Left-canonical gauge by successive Householder QR (FP64).

    A_k reshaped to (D_k d, D_{k+1}) = Q R with diag(R) >= 0; Q replaces A_k
    and R is absorbed into A_{k+1}.  The last R is the norm of the state: it
    is returned as its logarithm and the state is normalised.  Returns
    (sites, lognorm).
    """
    out = []
    carry = np.ones((1, 1))
    for k, a in enumerate(mps):
        a = tensordot(carry, a, [1], [0])              # [D_k, d, D_{k+1}]
        dk, d, dn = a.shape
        q, r = np.linalg.qr(a.reshape(dk * d, dn), mode="reduced")
        sgn = np.sign(np.diag(r))
        sgn[sgn == 0] = 1.0
        q = q * sgn[None, :]
        r = r * sgn[:, None]
        if q.shape[1] < dn:                            # rank-deficient width: keep shapes
            raise ValueError("bond larger than d*D_k is not supported")
        out.append(q.reshape(dk, d, dn))
        carry = r
    assert carry.shape == (1, 1)
    norm = float(carry[0, 0])
    return out, math.log(norm)


def env_left_step(l, a, w):
    """L_{k+1}[b', v, b] = sum A[a', t, b'] W[u, v, t, s] L_k[a', u, a] A[a, s, b]."""
    t1 = tensordot(l, a, [2], [0])                     # [a', u, s, b]
    t2 = tensordot(t1, w, [1, 2], [0, 3])              # [a', b, v, t]
    out = tensordot(a, t2, [0, 1], [0, 3])             # [b', b, v]
    return np.transpose(out, (0, 2, 1)).copy()         # [b', v, b]


def env_right_step(r, a, w):
    """R_k[a', u, a] = sum A[a', t, b'] W[u, v, t, s] R_{k+1}[b', v, b] A[a, s, b]."""
    t1 = tensordot(a, r, [2], [2])                     # [a, s, b', v]
    t2 = tensordot(t1, w, [1, 3], [3, 1])              # [a, b', u, t]
    out = tensordot(a, t2, [1, 2], [3, 1])             # [a', a, u]
    return np.transpose(out, (0, 2, 1)).copy()         # [a', u, a]


def env_sweep(psi, mpo, want_left=True, want_right=True):
    """Left and right environments of <psi|H|psi> and the energy from each side.

    L_0 = [[[1]]];  L_{k+1}[b', v, b] = sum A_k[a', t, b'] W_k[u, v, t, s] L_k[a', u, a] A_k[a, s, b]
    R_N = [[[1]]];  R_k[a', u, a]     = sum A_k[a', t, b'] W_k[u, v, t, s] R_{k+1}[b', v, b] A_k[a, s, b]
    E = L_N[0,0,0] = R_0[0,0,0].  Each step is three tensordots: the ket site
    into the environment, the MPO site, then the bra site.
    Returns (Ls, Rs, e_left, e_right).
    """
    n = len(psi)
    ls, rs = None, None
    e_left = e_right = None
    if want_left:
        ls = [np.ones((1, 1, 1))]
        for k in range(n):
            ls.append(env_left_step(ls[-1], psi[k], mpo[k]))
        e_left = float(ls[-1][0, 0, 0])
    if want_right:
        rs = [None] * (n + 1)
        rs[n] = np.ones((1, 1, 1))
        for k in range(n - 1, -1, -1):
            rs[k] = env_right_step(rs[k + 1], psi[k], mpo[k])
        e_right = float(rs[0][0, 0, 0])
    return ls, rs, e_left, e_right
