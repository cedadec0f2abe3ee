"""Oracle: pairwise contraction, trace, outer product and ncon networks (FP64).

Test infrastructure only (see the package docstring).

Definitions follow section III of the paper:
  * standard edge  -> a tensordot over the connected axes (III.A, "Standard Edges");
  * trace edge     -> the trace over the two axes of one node (III.A, "Trace Edges");
  * flattening     -> all edges between two nodes contracted as one (III.B, "Edge Flattening");
  * outer product  -> element-wise product of independent assignments (III.B, the outer-product equation);
  * ncon           -> label list per tensor, contraction in a given order (Appendix B).
"""
from __future__ import annotations

import numpy as np


def tensordot(a, b, axes_a, axes_b):
    """Sum over the paired axes (III.A "Standard Edges": numpy tensordot).

    Output axes: free axes of a in ascending order, then free axes of b in
    ascending order.  Computed as the definition itself states it: move the
    contracted axes to the inside, reshape to matrices, one matmul.
    """
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    axes_a = [int(x) % max(a.ndim, 1) for x in axes_a]
    axes_b = [int(x) % max(b.ndim, 1) for x in axes_b]
    if len(axes_a) != len(axes_b):
        raise ValueError("pair count mismatch")
    for i, j in zip(axes_a, axes_b):
        if a.shape[i] != b.shape[j]:
            raise ValueError("contracted dimensions differ")
    free_a = [i for i in range(a.ndim) if i not in axes_a]
    free_b = [j for j in range(b.ndim) if j not in axes_b]
    k = int(np.prod([a.shape[i] for i in axes_a], dtype=np.int64))
    am = np.transpose(a, free_a + axes_a).reshape(-1, k)
    bm = np.transpose(b, axes_b + free_b).reshape(k, -1)
    out_shape = tuple(a.shape[i] for i in free_a) + tuple(b.shape[j] for j in free_b)
    return np.matmul(am, bm).reshape(out_shape)


def contract_between(a, b, pairs):
    """contract_between (III.B): flatten every edge between a and b, then contract."""
    return tensordot(a, b, [p[0] for p in pairs], [p[1] for p in pairs])


def trace_edge(a, axis1, axis2):
    """Trace edge (III.A "Trace Edges"; the trace of Fig. 2): out[rest] = sum_i a[..i..i..].

    Remaining axes keep their ascending order.
    """
    a = np.asarray(a, dtype=np.float64)
    if axis1 == axis2 or a.shape[axis1] != a.shape[axis2]:
        raise ValueError("bad trace axes")
    rest = [i for i in range(a.ndim) if i not in (axis1, axis2)]
    moved = np.transpose(a, rest + [axis1, axis2])
    out = np.zeros(moved.shape[:-2])
    for i in range(a.shape[axis1]):
        out = out + moved[..., i, i]
    return out


def outer_product(a, b):
    """Outer product (III.B): (A (x) B)[i..., j...] = A[i...] * B[j...]."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return (a.reshape(-1, 1) * b.reshape(1, -1)).reshape(a.shape + b.shape)


def feature_map(p):
    """Local feature map of section IV.A: Phi(p) = (cos(pi p / 2), sin(pi p / 2))."""
    p = np.asarray(p, dtype=np.float64)
    return np.stack([np.cos(np.pi * p / 2.0), np.sin(np.pi * p / 2.0)], axis=-1)


def contract_network(tensors, labels, order=None):
    """ncon network (Appendix B) with the label convention used there.

    A label >= 0 names a connected edge and appears exactly twice (twice on
    one tensor = a trace edge); a label < 0 is a dangling edge and the output
    axes are ordered -1, -2, -3, ...  The edges are contracted in `order`
    (default: ascending labels).  When an edge joins two different nodes,
    every edge between those nodes is contracted with it (flattening, III.B);
    a self-edge is traced.  Nodes left unconnected at the end are combined by
    outer products in node order, then the result is permuted to the output
    order (reorder_edges).
    """
    nodes = [(np.asarray(t, dtype=np.float64), list(l)) for t, l in zip(tensors, labels)]
    for t, l in nodes:
        if t.ndim != len(l):
            raise ValueError("label count does not match rank")
    counts = {}
    for _, l in nodes:
        for x in l:
            counts[x] = counts.get(x, 0) + 1
    for x, c in counts.items():
        if x >= 0 and c != 2:
            raise ValueError(f"label {x} appears {c} times")
        if x < 0 and c != 1:
            raise ValueError(f"open label {x} repeated")
    if order is None:
        order = sorted(x for x in counts if x >= 0)
    done = set()
    for lab in order:
        if lab in done:
            continue
        where = [i for i, (_, l) in enumerate(nodes) if lab in l]
        if len(where) == 1:
            i = where[0]
            t, l = nodes[i]
            p = [j for j, x in enumerate(l) if x == lab]
            nt = trace_edge(t, p[0], p[1])
            nl = [x for j, x in enumerate(l) if j not in p]
            nodes[i] = (nt, nl)
            done.add(lab)
            continue
        i, j = where
        ti, li = nodes[i]
        tj, lj = nodes[j]
        shared = [x for x in li if x in lj]
        pairs = [(li.index(x), lj.index(x)) for x in shared]
        nt = contract_between(ti, tj, pairs)
        nl = [x for x in li if x not in shared] + [x for x in lj if x not in shared]
        done.update(shared)
        nodes = [n for k, n in enumerate(nodes) if k not in (i, j)] + [(nt, nl)]
    t, l = nodes[0]
    for t2, l2 in nodes[1:]:
        t = outer_product(t, t2)
        l = l + l2
    n_out = len(l)
    perm = [l.index(-(q + 1)) for q in range(n_out)]
    return np.transpose(t, perm).copy() if n_out else np.asarray(t)
