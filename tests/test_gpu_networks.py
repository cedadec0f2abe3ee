"""GPU parity of tree-like network contractions (TTN and binary MERA,
section II and section IV.B) against the FP64 oracle, contracted in the
order the library's own search returns (greedy, or exact for small
networks).  Norms are positive sums (gated relatively); expectation values
of operators of norm 1 are gated on the norm's scale (Cauchy-Schwarz)."""
import numpy as np
import pytest
import torch

import oracle
import paper_1905_01330_amd as tn
from helpers import greedy_order, random_orthogonal, report
from paper_1905_01330_amd import networks

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")
TOL = {"fp32": 1e-5, "split_bf16": 1e-6}
Z = np.diag([1.0, -1.0])
X = np.array([[0.0, 1.0], [1.0, 0.0]])


def state_tensors(n, chi, mera, seed, isometric=False):
    net, _ = networks.tree_state(n, 2, chi, mera)
    rng = np.random.default_rng(seed)
    out = []
    for kind, s in zip(net.kinds, net.shapes):
        if isometric and kind == "w":
            out.append(random_orthogonal(s[0] * s[1], rng)[:, :s[2]].reshape(s))
        elif isometric and kind == "u":
            out.append(random_orthogonal(s[0] * s[1], rng).reshape(s))
        elif isometric:
            r = rng.standard_normal(s)
            out.append(r / np.linalg.norm(r))
        else:
            out.append(rng.standard_normal(s) / np.sqrt(s[0] * s[1]))
    return [np.asarray(x, dtype=np.float32).astype(np.float64) for x in out]


def nodes_of(tensors, src, ops):
    it = iter([ops[k] for k in sorted(ops)])
    return [tensors[i] if i >= 0 else next(it) for i in src]


def run(n, chi, mera, ops, prec, method="greedy", seed=7, isometric=False):
    t = state_tensors(n, chi, mera, seed, isometric)
    shapes, labels, src = networks.expectation(n, 2, chi, tuple(sorted(ops)), mera)
    host = nodes_of(t, src, ops)
    dev = [torch.tensor(x, dtype=torch.float32, device=DEV) for x in host]
    order, flops = tn.network_order(dev, labels, method)
    got = float(tn.contract_network(dev, labels, order=order, prec=prec).cpu())
    ref = float(oracle.contract_network(host, labels, greedy_order(shapes, labels)))
    return got, ref, flops, host, labels, shapes


@pytest.mark.parametrize("mera", [False, True])
@pytest.mark.parametrize("prec", ["fp32", "split_bf16"])
def test_norm_and_local_expectations(mera, prec):
    n, chi = (32, 16) if not mera else (16, 8)
    got_n, ref_n, flops, *_ = run(n, chi, mera, {}, prec)
    assert abs(got_n - ref_n) <= TOL[prec] * ref_n, (got_n, ref_n)
    for ops in ({7: Z, 8: Z}, {5: X}, {0: Z, n - 1: Z}):
        got, ref, *_ = run(n, chi, mera, ops, prec)
        report(f"{'mera' if mera else 'ttn'}_expectation/{prec}", err_over_norm=abs(got - ref) / ref_n,
               order_flops=flops)
        assert abs(got - ref) <= TOL[prec] * ref_n, (ops, got, ref, ref_n)


def test_isometric_ttn_norm_is_one():
    got, _, flops, *_ = run(64, 32, False, {}, "split_bf16", isometric=True)
    assert abs(got - 1.0) <= 1e-6, got


def test_exact_order_on_a_small_network():
    for method in ("optimal", "greedy"):
        got, ref, flops, *_ = run(4, 4, False, {1: Z}, "fp32", method=method, seed=3)
        assert abs(got - ref) <= 1e-5 * abs(run(4, 4, False, {}, "fp32", method=method, seed=3)[1])


@pytest.mark.parametrize("prec", ["fp32", "split_bf16"])
@pytest.mark.parametrize("labels,spec", [
    ([[-1, 1, 2], [2, 1, -2]], "ijk,kjl->il"),    # two contracted axes whose strides do not merge
    ([[-1, 1, 2], [1, 2, -2]], "ijk,jkl->il"),    # the same pair merged into one axis
])
def test_k_sliced_network_steps(labels, spec, prec):
    """A step whose result is one or a few tiles (64 x 64) and whose contracted
    extent is long (4096) runs as k-slices of its outermost contracted axis,
    the partials summed in slice order.  FP32 accumulation over 4096 terms of
    unit variance: about u K / sqrt(2) absolute on entries up to about 4 sqrt(K)
    (split-BF16's six products accumulate in FP32 the same way), well inside
    5e-6 relative to the largest entry."""
    rng = np.random.default_rng(21)
    a = rng.standard_normal((64, 64, 64)).astype(np.float32)
    b = rng.standard_normal((64, 64, 64)).astype(np.float32)
    ref = np.einsum(spec, a.astype(np.float64), b.astype(np.float64))
    out = tn.contract_network([torch.tensor(a, device=DEV), torch.tensor(b, device=DEV)], labels, prec=prec)
    torch.cuda.synchronize()
    err = np.abs(out.cpu().double().numpy() - ref).max() / np.abs(ref).max()
    report(f"k-sliced network step {spec} {prec}", err=float(err))
    assert err <= 5e-6, err
