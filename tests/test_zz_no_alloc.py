"""tn_contract_network_noalloc (no workspace, static per-GPU scratch) against
tn_contract_network with a caller workspace, called through the C ABI.

Two calls in a row, the second on a smaller network, for a network whose
intermediates live in the scratch (one operator-environment step) and for
one whose split sums use it (a long dot product)."""
import ctypes as C

import numpy as np
import pytest
import torch

import oracle
import paper_1905_01330_amd as tn
from paper_1905_01330_amd import _lib as L
from paper_1905_01330_amd import inputs

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


def noalloc(tensors, labels, order, out, prec):
    flat, offs = [], [0]
    for lab in labels:
        flat.extend(lab)
        offs.append(len(flat))
    nodes = L.tensor_array(tensors)
    do = L.tensor_desc(out)
    L.check(L.lib().tn_contract_network_noalloc(len(tensors), nodes, L.int_array(flat), L.int_array(offs),
                                                len(order), L.int_array(order), C.byref(do), L.prec_code(prec),
                                                L.stream_ptr()))
    return out


def rel(a, b):
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


@pytest.mark.parametrize("prec", ["fp32", "split_bf16"])
def test_noalloc_environment_step_two_calls(prec):
    labels = [[1, 2, 3], [3, 4, -3], [2, -2, 5, 4], [1, 5, -1]]
    order = [3, 2, 4, 1, 5]
    tol = 1e-5 if prec == "fp32" else 1e-6
    for chi, seed in ((160, 1), (44, 2)):          # the second call is smaller
        rng = np.random.default_rng(seed)
        lk = rng.standard_normal((chi, 5, chi)).astype(np.float32)
        a = (rng.standard_normal((chi, 2, chi)) / np.sqrt(2 * chi)).astype(np.float32)
        w = inputs.xxz_mpo(3, 0.5)[1].astype(np.float32)
        host = [lk, a, w, a]
        dev = [torch.tensor(x, device=DEV) for x in host]
        ref = tn.contract_network(dev, labels, order=order, prec=prec)
        out = torch.full((chi, 5, chi), float("nan"), device=DEV)
        noalloc(dev, labels, order, out, prec)
        torch.cuda.synchronize()
        got, want = out.cpu().double().numpy(), ref.cpu().double().numpy()
        assert rel(got, want) <= tol, (chi, rel(got, want))
        assert rel(got, oracle.contract_network(host, labels, order)) <= tol


def test_noalloc_split_sum_two_calls():
    for n, seed in ((1 << 22, 3), (1 << 18, 4)):
        rng = np.random.default_rng(seed)
        x, y = rng.standard_normal(n).astype(np.float32), rng.standard_normal(n).astype(np.float32)
        dev = [torch.tensor(x, device=DEV), torch.tensor(y, device=DEV)]
        ref = tn.contract_network(dev, [[1], [1]], order=[1])
        out = torch.full((), float("nan"), device=DEV)
        noalloc(dev, [[1], [1]], [1], out, "fp32")
        torch.cuda.synchronize()
        exact = float(np.dot(x.astype(np.float64), y.astype(np.float64)))
        scale = float(np.dot(np.abs(x).astype(np.float64), np.abs(y).astype(np.float64)))
        assert abs(float(out.cpu()) - float(ref.cpu())) <= 1e-6 * scale
        assert abs(float(out.cpu()) - exact) <= 1e-6 * scale
