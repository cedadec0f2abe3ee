"""Oracle: complex tensors (FP64 complex128).

Test infrastructure only (see the package docstring).

The paper's node splitting writes V^dagger (section III.B), and physical
states are complex in general: contractions then carry complex products and
the bra of an inner product is conjugated.  Definitions:
  * pairwise contraction with optional conjugation of either node:
      C[free_a, free_b] = sum_k op_a(A)[.., k, ..] op_b(B)[.., k, ..],
    op = complex conjugation or identity (the tensordot of III.A otherwise);
  * MPS inner product <psi|phi> = sum_s conj(psi(s)) phi(s), by the same
    left-to-right recursion as the real case with psi's sites conjugated,
    rescaled by max|E| after every site (value m * exp(s), m complex).
"""
from __future__ import annotations

import math

import numpy as np


def tensordot_c(a, b, axes_a, axes_b, conj_a=False, conj_b=False):
    """Complex tensordot; output axes: free axes of a, then free axes of b."""
    a = np.asarray(a, dtype=np.complex128)
    b = np.asarray(b, dtype=np.complex128)
    if conj_a:
        a = np.conj(a)
    if conj_b:
        b = np.conj(b)
    axes_a = [int(x) % max(a.ndim, 1) for x in axes_a]
    axes_b = [int(x) % max(b.ndim, 1) for x in axes_b]
    for i, j in zip(axes_a, axes_b):
        if a.shape[i] != b.shape[j]:
            raise ValueError("contracted dimensions differ")
    free_a = [i for i in range(a.ndim) if i not in axes_a]
    free_b = [j for j in range(b.ndim) if j not in axes_b]
    k = int(np.prod([a.shape[i] for i in axes_a], dtype=np.int64))
    am = np.transpose(a, free_a + axes_a).reshape(-1, k)
    bm = np.transpose(b, axes_b + free_b).reshape(k, -1)
    shape = tuple(a.shape[i] for i in free_a) + tuple(b.shape[j] for j in free_b)
    return np.matmul(am, bm).reshape(shape)


def mps_inner_c(psi, phi):
    """<psi|phi> for complex MPS sites [D_k, d, D_{k+1}]: (m, s) with value m * exp(s)."""
    e = np.ones((1, 1), dtype=np.complex128)
    logs = 0.0
    for a, b in zip(psi, phi):
        t = tensordot_c(e, b, [1], [0])                     # [a', s, b]
        e = tensordot_c(a, t, [0, 1], [0, 1], conj_a=True)  # [b', b]
        mx = float(np.max(np.abs(e)))
        if mx > 0 and np.isfinite(mx):
            e = e / mx
            logs += math.log(mx)
    return complex(e[0, 0]), logs


def mps_to_dense_c(mps):
    """Dense amplitudes (site 0 most significant) of a complex MPS."""
    n = len(mps)
    d = mps[0].shape[1]
    idx = np.arange(d ** n)
    digits = [(idx // d ** (n - 1 - k)) % d for k in range(n)]
    acc = np.asarray(mps[0], dtype=np.complex128)[0, digits[0], :][:, None, :]
    for k in range(1, n):
        mats = np.transpose(np.asarray(mps[k], dtype=np.complex128), (1, 0, 2))[digits[k]]
        acc = np.matmul(acc, mats)
    return acc[:, 0, 0]
