"""Oracle: node splitting by singular value decomposition, with truncation (FP64).

Test infrastructure only (see the package docstring).

Section III.B "Node Splitting": the legs of a node are grouped into a left
and a right effective leg, the node is read as the matrix A[(left), (right)]
and decomposed as A = U S V^dagger (real arithmetic here, so V^dagger = V^T).
The new bond has dimension min(prod left dims, prod right dims) before any
truncation.  split_node returns the two factors with the square root of the
singular values absorbed into each (U sqrt(S), sqrt(S) V^T);
split_node_full_svd returns U, S (a diagonal matrix node) and V^T.

Appendix A "Saving Memory": the smallest singular values may be dropped,
either keeping at most `max_singular_values` of them or dropping the largest
set of smallest values whose sum does not exceed `max_truncation_err` (the
paper states the bound on the values adding up).  With both limits the
smaller rank wins.  At least one value is kept: a bond of dimension zero is
not a tensor.  The dropped values, largest first, are returned as trun_err.

numpy's SVD is the library step; everything else is written out here.
"""
from __future__ import annotations

import numpy as np


def truncation_rank(s, max_singular_values=None, max_truncation_err=None):
    """Number of singular values kept, for s sorted in descending order.

    k_count = min(len(s), max_singular_values); k_err = the smallest k such
    that sum(s[k:]) <= max_truncation_err; the result is max(1, min of the
    two)."""
    s = np.asarray(s, dtype=np.float64)
    n = len(s)
    k = n
    if max_singular_values is not None:
        k = min(k, int(max_singular_values))
    if max_truncation_err is not None:
        # dropped[j] = sum of s[j:], the sum left out when j values are kept
        dropped = np.concatenate([np.cumsum(s[::-1])[::-1], [0.0]])
        k_err = int(np.argmax(dropped <= max_truncation_err))
        k = min(k, k_err)
    return max(1, k)


def svd_matrix(a, n_left):
    """The matrix of section III.B: legs 0..n_left-1 form the rows, the rest
    the columns; returns (matrix, left dims, right dims)."""
    a = np.asarray(a, dtype=np.float64)
    left, right = a.shape[:n_left], a.shape[n_left:]
    m = int(np.prod(left, dtype=np.int64))
    n = int(np.prod(right, dtype=np.int64))
    return a.reshape(m, n), tuple(left), tuple(right)


def split_node_full_svd(a, n_left, max_singular_values=None, max_truncation_err=None):
    """(U, S, V^T, trun_err): U has shape left + (k,), S is (k, k) diagonal,
    V^T has shape (k,) + right, trun_err holds the dropped singular values."""
    mat, left, right = svd_matrix(a, n_left)
    u, s, vt = np.linalg.svd(mat, full_matrices=False)
    k = truncation_rank(s, max_singular_values, max_truncation_err)
    trun = s[k:].copy()
    return (u[:, :k].reshape(left + (k,)), np.diag(s[:k]), vt[:k].reshape((k,) + right), trun)


def split_node(a, n_left, max_singular_values=None, max_truncation_err=None):
    """(U sqrt(S), sqrt(S) V^T, trun_err) with the same truncation."""
    u, s, vt, trun = split_node_full_svd(a, n_left, max_singular_values, max_truncation_err)
    r = np.sqrt(np.diag(s))                       # sqrt of the kept singular values
    left = u * r                                  # scales the last axis (the new bond)
    right = r.reshape((-1,) + (1,) * (vt.ndim - 1)) * vt   # scales the first axis
    return left, right, trun
