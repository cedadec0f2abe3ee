"""Network structures of the paper's tree-like states (section II, the
overview figure of MPS, TTN and MERA; section IV.B, the TTN ground-state
computation): label lists in the ncon convention of Appendix B (a label >= 0
is a connected edge, < 0 a dangling one, outputs -1, -2, ...).

This module only lays out structure (which legs connect, their extents);
there is no arithmetic here.  The tensors are supplied by the caller, one per
node, with the shapes listed.

Binary tree tensor network (TTN) on n = 2^L sites of dimension d: level 1
holds n/2 isometries w[lower1, lower2, upper] joining pairs of sites, level
l joins pairs of level l-1 bonds; the top is a root [left, right].  The bond
above level l has extent min(chi, d^(2^l)).

Binary MERA: every level first applies disentanglers u[lower1, lower2,
upper1, upper2] to the pairs of positions (2j+1, 2j+2) (open boundary: no
disentangler on the ends), then isometries w[lower1, lower2, upper] to the
pairs (2j, 2j+1); the top is a root over the last two positions.
"""
from __future__ import annotations


class Net:
    """A state network: node shapes, labels per node, and the kind of each
    node ("w", "u", "root"); physical legs carry the labels phys[i]."""

    def __init__(self):
        self.shapes, self.labels, self.kinds = [], [], []

    def add(self, kind, shape, labels):
        self.shapes.append(tuple(int(x) for x in shape))
        self.labels.append([int(x) for x in labels])
        self.kinds.append(kind)


def _bond(d, chi, level):
    v = d
    for _ in range(level):
        v = v * v
        if v >= chi:
            return chi
    return min(chi, v)


def tree_state(n_sites, d, chi, mera=False, phys=None, first_label=None):
    """The TTN (mera=False) or binary MERA (mera=True) state with physical
    labels phys[i] (default: -(i+1), all open).  Internal labels start at
    first_label (default: max(phys)+1, or 1) and are numbered from the
    bottom up.  Returns (Net, next free label)."""
    if n_sites < 2 or n_sites & (n_sites - 1):
        raise ValueError("n_sites must be a power of two >= 2")
    phys = list(phys) if phys is not None else [-(i + 1) for i in range(n_sites)]
    nxt = first_label if first_label is not None else max([x + 1 for x in phys if x >= 0] + [1])
    net = Net()
    cur = list(phys)                      # label of the open leg above each position
    dims = [d] * n_sites
    level = 0
    while len(cur) > 2:
        level += 1
        if mera:
            for j in range(0, len(cur) // 2 - 1):
                a, b = 2 * j + 1, 2 * j + 2
                up = [nxt, nxt + 1]
                nxt += 2
                net.add("u", (dims[a], dims[b], dims[a], dims[b]), [cur[a], cur[b], up[0], up[1]])
                cur[a], cur[b] = up
        nd = _bond(d, chi, level)
        new, newdims = [], []
        for j in range(len(cur) // 2):
            a, b = 2 * j, 2 * j + 1
            net.add("w", (dims[a], dims[b], nd), [cur[a], cur[b], nxt])
            new.append(nxt)
            newdims.append(nd)
            nxt += 1
        cur, dims = new, newdims
    net.add("root", (dims[0], dims[1]), [cur[0], cur[1]])
    return net, nxt


def expectation(n_sites, d, chi, ops=(), mera=False):
    """<psi| O |psi> with O a product of one-site operators op[s_bra, s_ket]
    on the sites listed in `ops`: the ket network, one node per operator and
    the bra network (the same tensors, relabelled).  Returns (shapes, labels,
    node -> index of the state tensor it uses, or -1 for an operator node);
    every label is connected, so the result is a scalar."""
    ket_phys = list(range(1, n_sites + 1))
    bra_phys = list(ket_phys)
    op_nodes = []
    nxt = n_sites + 1
    for site in ops:
        bra_phys[site] = nxt
        op_nodes.append((site, nxt, ket_phys[site]))
        nxt += 1
    ket, nxt = tree_state(n_sites, d, chi, mera, ket_phys, nxt)
    bra, nxt = tree_state(n_sites, d, chi, mera, bra_phys, nxt)
    shapes = list(ket.shapes)
    labels = [list(x) for x in ket.labels]
    src = list(range(len(ket.shapes)))
    for site, lb, lk in op_nodes:
        shapes.append((d, d))
        labels.append([lb, lk])
        src.append(-1)
    shapes += bra.shapes
    labels += [list(x) for x in bra.labels]
    src += list(range(len(bra.shapes)))
    return shapes, labels, src
