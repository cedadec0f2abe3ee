"""Pins of the oracle's MPS inner product, canonicalisation and environment sweep.

Independent routes: dense state vectors built amplitude by amplitude, dense
Hamiltonians from Pauli strings, exact diagonalisation, the closed-form
ground energies of the critical transverse-field Ising chain and of the XX
chain, and product states with known norms and energies hidden by random
orthogonal gauges.
"""
import math

import numpy as np
import pytest

import oracle
from helpers import (
    dense_tfim,
    dense_to_mps,
    dense_xxz,
    product_state_mps,
    rel_fro,
    spin_angle_vector,
    tfim_ground_energy_closed_form,
    xx_ground_energy_closed_form,
)
from paper_1905_01330_amd import inputs


def test_dense_state_builder_pins():
    # a product state's dense vector is the Kronecker product of its local vectors
    rng = np.random.default_rng(1)
    vs = [rng.standard_normal(2) for _ in range(5)]
    sites = [v.reshape(1, 2, 1) for v in vs]
    ref = vs[0]
    for v in vs[1:]:
        ref = np.kron(ref, v)
    np.testing.assert_allclose(oracle.mps_to_dense(sites), ref, rtol=1e-14)


def test_inner_cfg1_matches_dense_state_vectors():
    # N = 16, d = 2, chi = 16, independent psi and phi (seeds 101, 102)
    psi = inputs.random_mps(16, 2, 16, 101)
    phi = inputs.random_mps(16, 2, 16, 102)
    dpsi, dphi = oracle.mps_to_dense(psi), oracle.mps_to_dense(phi)
    m, s = oracle.mps_inner(psi, phi)
    val = m * math.exp(s)
    ref = float(np.dot(dpsi, dphi))
    cs = np.linalg.norm(dpsi) * np.linalg.norm(dphi)
    assert abs(val - ref) / cs <= 1e-12
    for x in (psi, phi):
        mm, ss = oracle.mps_inner(x, x)
        dn = float(np.dot(oracle.mps_to_dense(x), oracle.mps_to_dense(x)))
        assert abs(mm * math.exp(ss) / dn - 1.0) <= 1e-12


def test_inner_left_equals_right():
    from oracle.mps import mps_inner_right
    psi, phi = inputs.correlated_mps_pair(20, 2, 12, 5)
    m1, s1 = oracle.mps_inner(psi, phi)
    m2, s2 = mps_inner_right(psi, phi)
    assert abs(m1 * math.exp(s1 - s2) / m2 - 1.0) < 1e-12


def test_inner_norm_positive_and_rescaling_consistent():
    psi = inputs.random_mps(40, 2, 32, 8)
    m, s = oracle.mps_inner(psi, psi)
    assert m > 0
    m0, s0 = oracle.mps_inner(psi, psi, rescale=False)
    assert s0 == 0.0
    assert abs(m * math.exp(s) / m0 - 1.0) < 1e-12


@pytest.mark.parametrize("chi", [1, 8, 32])
def test_normalised_product_state_has_norm_one(chi):
    rng = np.random.default_rng(40 + chi)
    n = 24
    vecs = []
    for _ in range(n):
        v = rng.standard_normal(2)
        vecs.append(v / np.linalg.norm(v))
    dims = inputs.bond_dims(n, 2, chi)
    sites = product_state_mps(vecs, dims, rng)
    m, s = oracle.mps_inner(sites, sites)
    assert abs(m * math.exp(s) - 1.0) < 1e-12


def test_mpo_matches_pauli_hamiltonians():
    for n in (2, 3, 5):
        np.testing.assert_allclose(oracle.mpo_to_dense(inputs.tfim_mpo(n, 1.0, 0.7)), dense_tfim(n, 1.0, 0.7), atol=1e-13)
        np.testing.assert_allclose(oracle.mpo_to_dense(inputs.xxz_mpo(n, 0.5)), dense_xxz(n, 0.5), atol=1e-13)


def test_closed_forms_against_exact_diagonalisation():
    for n in (2, 4, 7, 9):
        e = np.linalg.eigvalsh(dense_tfim(n))[0]
        assert abs(e - tfim_ground_energy_closed_form(n)) < 1e-11
        e = np.linalg.eigvalsh(dense_xxz(n, 0.0))[0]
        assert abs(e - xx_ground_energy_closed_form(n)) < 1e-11


def test_env_energy_matches_dense_expectation():
    n = 9
    psi = inputs.random_mps(n, 2, 8, 17)
    for mpo, h in ((inputs.tfim_mpo(n), dense_tfim(n)), (inputs.xxz_mpo(n, 0.5), dense_xxz(n, 0.5))):
        _, _, el, er = oracle.env_sweep(psi, mpo)
        v = oracle.mps_to_dense(psi)
        ref = float(v @ h @ v)
        assert abs(el - ref) <= 1e-12 * max(1.0, abs(ref))
        assert abs(er - ref) <= 1e-12 * max(1.0, abs(ref))


def test_env_sweep_tfim_ground_state_closed_form():
    n = 10
    w, vecs = np.linalg.eigh(dense_tfim(n))
    sites = dense_to_mps(vecs[:, 0], n)
    _, _, el, er = oracle.env_sweep(sites, inputs.tfim_mpo(n))
    e0 = tfim_ground_energy_closed_form(n)
    assert abs(el - e0) < 1e-10 and abs(er - e0) < 1e-10


def test_env_sweep_xx_ground_state_closed_form():
    n = 8
    w, vecs = np.linalg.eigh(dense_xxz(n, 0.0))
    sites = dense_to_mps(vecs[:, 0], n)
    _, _, el, _ = oracle.env_sweep(sites, inputs.xxz_mpo(n, 0.0))
    assert abs(el - xx_ground_energy_closed_form(n)) < 1e-10


def test_env_sweep_product_states_closed_forms():
    rng = np.random.default_rng(55)
    n, chi = 30, 16
    dims = inputs.bond_dims(n, 2, chi)
    th = rng.uniform(0, 2 * np.pi, n)
    sites = product_state_mps([spin_angle_vector(t) for t in th], dims, rng)
    J, g = 1.0, 0.8
    ref = -J * sum(math.cos(th[i]) * math.cos(th[i + 1]) for i in range(n - 1)) - g * sum(math.sin(t) for t in th)
    _, _, el, er = oracle.env_sweep(sites, inputs.tfim_mpo(n, J, g))
    assert abs(el - ref) < 1e-11 and abs(er - ref) < 1e-11
    delta = 0.5
    up, dn = np.array([1.0, 0.0]), np.array([0.0, 1.0])
    allup = product_state_mps([up] * n, dims, rng)
    neel = product_state_mps([up if i % 2 == 0 else dn for i in range(n)], dims, rng)
    _, _, e1, _ = oracle.env_sweep(allup, inputs.xxz_mpo(n, delta))
    _, _, e2, _ = oracle.env_sweep(neel, inputs.xxz_mpo(n, delta))
    assert abs(e1 - delta * (n - 1) / 4) < 1e-11
    assert abs(e2 + delta * (n - 1) / 4) < 1e-11


def test_canonical_form_isometry_and_state():
    n, chi = 12, 16
    raw = inputs.random_mps(n, 2, chi, 201)
    can, lognorm = oracle.left_canonicalize(raw)
    for a in can:
        dk, d, dn = a.shape
        m = a.reshape(dk * d, dn)
        np.testing.assert_allclose(m.T @ m, np.eye(dn), atol=1e-13)
    v_raw, v_can = oracle.mps_to_dense(raw), oracle.mps_to_dense(can)
    nrm = np.linalg.norm(v_raw)
    assert abs(math.log(nrm) - lognorm) < 1e-12
    np.testing.assert_allclose(v_can, v_raw / nrm, atol=1e-12)
    # same factorisation as numpy's QR route with the diag(R) >= 0 convention
    q, r = np.linalg.qr(raw[0].reshape(2, -1))
    q = q * np.sign(np.diag(r))[None, :]
    np.testing.assert_allclose(can[0].reshape(2, -1), q, atol=1e-14)


def test_env_identity_channel_and_cut_invariance():
    n, chi = 14, 16
    psi, _ = oracle.left_canonicalize(inputs.random_mps(n, 2, chi, 201))
    mpo = inputs.tfim_mpo(n)
    ls, rs, el, er = oracle.env_sweep(psi, mpo)
    for k in range(1, n):
        np.testing.assert_allclose(ls[k][:, 0, :], np.eye(ls[k].shape[0]), atol=1e-12)
    for k in range(n + 1):
        cut = float(np.sum(ls[k] * rs[k]))
        assert abs(cut - el) < 1e-11 * max(1, abs(el))
    assert abs(el - er) < 1e-11 * max(1, abs(el))


def test_bond_dims():
    assert inputs.bond_dims(16, 2, 16) == [1, 2, 4, 8, 16, 16, 16, 16, 16, 16, 16, 16, 16, 8, 4, 2, 1]
    dims = inputs.bond_dims(64, 2, 1024)
    assert max(dims) == 1024 and dims[0] == dims[-1] == 1 and dims.count(1024) == 45
