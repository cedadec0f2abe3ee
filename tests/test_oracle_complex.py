"""Pins of the complex oracle: brute-force index loops for the conjugated
contractions, the dense state vector (numpy's vdot conjugates its first
argument) for inner products, and the symmetries <psi|psi> > 0 and
<psi|phi> = conj(<phi|psi>)."""
import itertools
import math

import numpy as np
import pytest

import oracle
from paper_1905_01330_amd import inputs


def brute(a, b, axes_a, axes_b, ca, cb):
    a = np.conj(a) if ca else a
    b = np.conj(b) if cb else b
    free_a = [i for i in range(a.ndim) if i not in axes_a]
    free_b = [j for j in range(b.ndim) if j not in axes_b]
    out = np.zeros([a.shape[i] for i in free_a] + [b.shape[j] for j in free_b], dtype=complex)
    for o in itertools.product(*[range(s) for s in out.shape]):
        acc = 0j
        for k in itertools.product(*[range(a.shape[i]) for i in axes_a]):
            ia, ib = [0] * a.ndim, [0] * b.ndim
            for p, i in enumerate(free_a):
                ia[i] = o[p]
            for p, j in enumerate(free_b):
                ib[j] = o[len(free_a) + p]
            for p, (i, j) in enumerate(zip(axes_a, axes_b)):
                ia[i] = ib[j] = k[p]
            acc += a[tuple(ia)] * b[tuple(ib)]
        out[o] = acc
    return out


@pytest.mark.parametrize("seed", range(8))
def test_tensordot_c_against_loops(seed):
    rng = np.random.default_rng(seed)
    a = rng.standard_normal((3, 2, 4)) + 1j * rng.standard_normal((3, 2, 4))
    b = rng.standard_normal((4, 3, 2)) + 1j * rng.standard_normal((4, 3, 2))
    ca, cb = bool(seed & 1), bool(seed & 2)
    for axes_a, axes_b in (([2], [0]), ([0, 2], [1, 0]), ([], [])):
        got = oracle.tensordot_c(a, b, axes_a, axes_b, ca, cb)
        np.testing.assert_allclose(got, brute(a, b, axes_a, axes_b, ca, cb), atol=1e-12)


def test_inner_product_matches_dense_vdot():
    psi = inputs.random_mps_complex(10, 2, 8, 1)
    phi = inputs.random_mps_complex(10, 2, 8, 2)
    m, s = oracle.mps_inner_c(psi, phi)
    want = np.vdot(oracle.mps_to_dense_c(psi), oracle.mps_to_dense_c(phi))
    assert abs(m * math.exp(s) - want) <= 1e-12 * abs(want)
    mr, sr = oracle.mps_inner_c(phi, psi)
    assert abs(mr * math.exp(sr) - np.conj(want)) <= 1e-12 * abs(want)
    mn, sn = oracle.mps_inner_c(psi, psi)
    assert mn.real > 0 and abs(mn.imag) <= 1e-14 * abs(mn)


def test_real_sites_reduce_to_the_real_inner_product():
    psi = inputs.random_mps(12, 2, 8, 3)
    phi = inputs.random_mps(12, 2, 8, 4)
    m, s = oracle.mps_inner_c(psi, phi)
    mr, sr = oracle.mps_inner(psi, phi)
    assert abs(m.imag) == 0.0 and abs(m.real * math.exp(s) - mr * math.exp(sr)) <= 1e-12 * abs(mr * math.exp(sr))
