"""GPU parity of the two-site DMRG update against the FP64 oracle: the
effective-Hamiltonian mat-vec, the Lanczos eigenpair, the update with its
split, and whole sweeps against closed-form ground energies.

Environments come from random canonical MPS (oracle-built on the host), so
H_eff is the projection of a real Hamiltonian.  Eigenvectors are compared
through |<theta, theta_ref>| (the sign is not fixed)."""
import numpy as np
import pytest
import torch

import oracle
import paper_1905_01330_amd as tn
from helpers import report, tfim_ground_energy_closed_form, xx_ground_energy_closed_form
from paper_1905_01330_amd import inputs

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")
TOL = {"fp32": 1e-5, "split_bf16": 1e-6}


def r32(x):
    return np.asarray(x, dtype=np.float32).astype(np.float64)


def g32(x):
    return torch.tensor(np.asarray(x, dtype=np.float32), device=DEV)


def environments(n, chi, k, model, seed):
    """L_k from left-canonical sites < k, R_{k+2} from right-canonical sites > k+1."""
    mpo = inputs.tfim_mpo(n) if model == "tfim" else inputs.xxz_mpo(n, 0.5)
    raw = inputs.random_mps(n, 2, chi, seed)
    left, _ = oracle.left_canonicalize(raw)
    mirrored, _ = oracle.left_canonicalize([np.transpose(a, (2, 1, 0)) for a in reversed(raw)])
    right = [np.transpose(a, (2, 1, 0)) for a in reversed(mirrored)]
    l = np.ones((1, 1, 1))
    for j in range(k):
        l = oracle.env_left_step(l, left[j], mpo[j])
    r = np.ones((1, 1, 1))
    for j in range(n - 1, k + 1, -1):
        r = oracle.env_right_step(r, right[j], mpo[j])
    return r32(l), r32(r), r32(mpo[k]), r32(mpo[k + 1])


@pytest.mark.parametrize("prec", ["fp32", "split_bf16"])
def test_heff_matvec(prec):
    l, r, w1, w2 = environments(14, 48, 6, "xxz", 3)
    th = r32(np.random.default_rng(1).standard_normal((l.shape[0], 2, 2, r.shape[0])))
    got = tn.dmrg_apply_heff(g32(l), g32(r), g32(w1), g32(w2), g32(th), prec=prec).cpu().double().numpy()
    ref = oracle.heff_apply(l, r, w1, w2, th)
    err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    report(f"dmrg_heff/{prec}", rel_err=err)
    assert err <= TOL[prec], err


@pytest.mark.parametrize("model", ["tfim", "xxz"])
def test_eigensolve_vs_dense(model):
    l, r, w1, w2 = environments(12, 8, 5, model, 11)
    h = oracle.heff_dense(l, r, w1, w2)
    vals, vecs = np.linalg.eigh(0.5 * (h + h.T))
    th = g32(np.random.default_rng(2).standard_normal((l.shape[0], 2, 2, r.shape[0])))
    out = tn.dmrg_eigensolve(g32(l), g32(r), g32(w1), g32(w2), th, krylov=24, restarts=4).cpu().numpy()
    got = th.cpu().double().numpy().ravel()
    ov = abs(float(got @ vecs[:, 0]))
    report(f"dmrg_eigensolve/{model}", energy_rel_err=abs(out[0] - vals[0]) / abs(vals[0]), overlap=ov,
           residual=float(out[1]))
    assert abs(out[0] - vals[0]) <= 1e-5 * abs(vals[0]), (out, vals[:3])
    assert abs(np.linalg.norm(got) - 1.0) < 1e-6 and ov >= 1 - 1e-5, ov
    assert out[1] <= 1e-4 * abs(vals[0])


def test_small_space_breakdown():
    """At the chain's end the two-site space has 8 states, fewer than the
    Krylov vectors: the recursion stops at the invariant subspace."""
    l, r, w1, w2 = environments(10, 8, 0, "tfim", 13)
    h = oracle.heff_dense(l, r, w1, w2)
    assert h.shape[0] < 24
    vals = np.linalg.eigvalsh(0.5 * (h + h.T))
    th = g32(np.random.default_rng(3).standard_normal((l.shape[0], 2, 2, r.shape[0])))
    out = tn.dmrg_eigensolve(g32(l), g32(r), g32(w1), g32(w2), th, krylov=24, restarts=2).cpu().numpy()
    assert np.isfinite(out).all() and abs(out[0] - vals[0]) <= 1e-5 * abs(vals[0]), (out, vals)


def test_two_site_update_vs_oracle():
    l, r, w1, w2 = environments(12, 8, 4, "xxz", 17)
    e_ref, th_ref, a_ref, b_ref, tr_ref = oracle.two_site_update(l, r, w1, w2, chi_max=6, direction="right")
    th = g32(np.random.default_rng(4).standard_normal(th_ref.shape))
    out2, a, b, tr = tn.dmrg_two_site_update(g32(l), g32(r), g32(w1), g32(w2), th, chi_max=6, restarts=4)
    e = float(out2[0].cpu())
    assert abs(e - e_ref) <= 1e-5 * abs(e_ref)
    assert tuple(a.shape) == a_ref.shape and tuple(b.shape) == b_ref.shape and tuple(tr.shape) == tr_ref.shape
    np.testing.assert_allclose(tr.cpu().double().numpy(), tr_ref, atol=1e-5)
    am = a.cpu().double().numpy().reshape(-1, a.shape[2])
    np.testing.assert_allclose(am.T @ am, np.eye(am.shape[1]), atol=1e-6)
    prod = np.tensordot(a.cpu().double().numpy(), b.cpu().double().numpy(), 1)
    prod_ref = np.tensordot(a_ref, b_ref, 1)
    assert abs(abs(float(np.sum(prod * prod_ref))) - float(np.sum(prod_ref * prod_ref))) <= 1e-5


def start_state(n, chi, seed):
    sites = [torch.tensor(x, device=DEV) for x in inputs.random_mps(n, 2, chi, seed)]
    tn.mps_left_canonicalize(sites)
    return [s.float().contiguous() for s in sites]


@pytest.mark.parametrize("n", [16, 24])
def test_dmrg_critical_ising_closed_form(n):
    mpo = [g32(x) for x in inputs.tfim_mpo(n)]
    energies, psi = tn.dmrg(mpo, start_state(n, 4, 21), chi_max=32, sweeps=3)
    e0 = tfim_ground_energy_closed_form(n)
    err = abs(energies[-1] - e0) / abs(e0)
    report(f"dmrg_tfim/N{n}", energy=energies[-1], exact=e0, rel_err=err)
    assert err <= 1e-5, (energies[-1], e0)
    assert max(psi[k].shape[2] for k in range(n - 1)) <= 32


def test_dmrg_xx_closed_form():
    n = 16
    mpo = [g32(x) for x in inputs.xxz_mpo(n, 0.0)]
    energies, _ = tn.dmrg(mpo, start_state(n, 4, 23), chi_max=32, sweeps=3)
    e0 = xx_ground_energy_closed_form(n)
    report("dmrg_xx/N16", energy=energies[-1], exact=e0, rel_err=abs(energies[-1] - e0) / abs(e0))
    assert abs(energies[-1] - e0) <= 1e-5 * abs(e0), (energies[-1], e0)
