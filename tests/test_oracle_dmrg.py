"""Pins of the two-site DMRG oracle: the effective Hamiltonian equals the
dense Hamiltonian projected through the MPS bases of the other sites, and
sweeps reach energies known in closed form (critical transverse-field Ising
chain, XX chain) or by exact diagonalisation."""
import numpy as np
import pytest

import oracle
from oracle.dmrg import dmrg, heff_apply, heff_dense, two_site_update
from helpers import dense_tfim, dense_xxz, tfim_ground_energy_closed_form, xx_ground_energy_closed_form
from paper_1905_01330_amd import inputs


def right_canonical(mps):
    """Right-canonical gauge (every site k > 0 satisfies sum_s B^s B^s^T = I) by
    left-canonicalising the mirrored chain."""
    mirrored = [np.transpose(a, (2, 1, 0)) for a in reversed(mps)]
    can, lognorm = oracle.left_canonicalize(mirrored)
    return [np.transpose(a, (2, 1, 0)) for a in reversed(can)]


def left_block(sites):
    """[d^k, D_k]: amplitudes of the left sites as vectors of the bond (k >= 1)."""
    acc = sites[0].reshape(-1, sites[0].shape[2])            # [s0, D1]
    for a in sites[1:]:
        acc = np.tensordot(acc, a, axes=([1], [0])).reshape(-1, a.shape[2])
    return acc


def right_block(sites):
    """[D, d^m]: amplitudes of the right sites as vectors of the bond."""
    acc = sites[-1].reshape(sites[-1].shape[0], -1)          # [D, s]
    for a in reversed(sites[:-1]):
        acc = np.tensordot(a, acc, axes=([2], [0])).reshape(a.shape[0], -1)
    return acc


@pytest.mark.parametrize("model", ["tfim", "xxz"])
@pytest.mark.parametrize("k", [0, 2, 4])
def test_effective_hamiltonian_is_the_projected_hamiltonian(model, k):
    n, chi = 6, 4
    mpo = inputs.tfim_mpo(n, 1.0, 0.7) if model == "tfim" else inputs.xxz_mpo(n, 0.6)
    h = dense_tfim(n, 1.0, 0.7) if model == "tfim" else dense_xxz(n, 0.6)
    raw = inputs.random_mps(n, 2, chi, 31 + k)
    left, _ = oracle.left_canonicalize(raw)                  # sites < k left-canonical
    right = right_canonical(raw)                             # sites > k+1 right-canonical
    l = np.ones((1, 1, 1))
    for j in range(k):
        l = oracle.env_left_step(l, left[j], mpo[j])
    r = np.ones((1, 1, 1))
    for j in range(n - 1, k + 1, -1):
        r = oracle.env_right_step(r, right[j], mpo[j])
    dl, dr = left[k].shape[0] if k > 0 else 1, right[k + 1].shape[2] if k + 2 < n else 1
    lb = left_block(left[:k]) if k > 0 else np.ones((1, 1))           # [d^k, dl]
    rb = right_block(right[k + 2:]) if k + 2 < n else np.ones((1, 1))  # [dr, d^m]
    # P maps theta[a, s1, s2, b] to the dense state sum_ab lb[sL, a] theta rb[b, sR]
    p = np.einsum("xa,st,uv,by->xsuyatvb", lb, np.eye(2), np.eye(2), rb).reshape(2 ** n, dl * 4 * dr)
    want = p.T @ h @ p
    got = heff_dense(l, r, mpo[k], mpo[k + 1])
    np.testing.assert_allclose(got, want, atol=1e-12 * max(1.0, np.abs(want).max()))
    # and the mat-vec form agrees with the dense matrix
    th = np.random.default_rng(k).standard_normal((dl, 2, 2, dr))
    np.testing.assert_allclose(heff_apply(l, r, mpo[k], mpo[k + 1], th).ravel(), got @ th.ravel(), atol=1e-12)


def test_two_site_update_properties():
    n, chi = 8, 8
    mpo = inputs.tfim_mpo(n)
    psi = right_canonical(inputs.random_mps(n, 2, chi, 5))
    r = np.ones((1, 1, 1))
    for j in range(n - 1, 1, -1):
        r = oracle.env_right_step(r, psi[j], mpo[j])
    e, theta, a, b, trun = two_site_update(np.ones((1, 1, 1)), r, mpo[0], mpo[1], chi_max=2)
    assert abs(np.linalg.norm(theta) - 1.0) < 1e-12
    rq = float(np.sum(theta * heff_apply(np.ones((1, 1, 1)), r, mpo[0], mpo[1], theta)))
    assert abs(rq - e) < 1e-12 * max(1.0, abs(e))
    am = a.reshape(-1, a.shape[2])
    np.testing.assert_allclose(am.T @ am, np.eye(am.shape[1]), atol=1e-12)   # left-canonical
    assert a.shape[2] == 2 and b.shape[0] == 2 and len(trun) == 0             # a 1*2 x 2*D matrix has rank 2


@pytest.mark.parametrize("n", [8, 10])
def test_dmrg_reaches_the_critical_ising_closed_form(n):
    psi0 = right_canonical(inputs.random_mps(n, 2, 4, 7))
    energies, _ = dmrg(inputs.tfim_mpo(n), psi0, chi_max=16, sweeps=2)
    e0 = tfim_ground_energy_closed_form(n)
    assert abs(energies[-1] - e0) < 1e-8 * abs(e0), (energies[-1], e0)
    if n == 8:
        assert abs(e0 - np.linalg.eigvalsh(dense_tfim(n))[0]) < 1e-10


def test_dmrg_reaches_the_xx_closed_form():
    n = 8
    psi0 = right_canonical(inputs.random_mps(n, 2, 4, 9))
    energies, _ = dmrg(inputs.xxz_mpo(n, 0.0), psi0, chi_max=16, sweeps=2)
    want = xx_ground_energy_closed_form(n)
    assert abs(want - float(np.linalg.eigvalsh(dense_xxz(n, 0.0))[0])) < 1e-10
    assert abs(energies[-1] - want) < 1e-8 * abs(want), (energies[-1], want)
