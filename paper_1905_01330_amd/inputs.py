"""Seeded synthetic inputs shared by the GPU path, the tests and the benchmark.

This module only draws random numbers and lays out model constants (the
Pauli matrices of the spin-chain operators).  It performs none of the
contraction arithmetic: neither side's result is computed here.  Arrays are
float64 on the host (the uneven-batch chains are float32, see uneven_chain);
callers cast and upload as they need.

Layouts (shared by every consumer):
  * MPS site k:  A_k[D_k, d, D_{k+1}], open boundaries D_0 = D_N = 1.
  * MPO site k:  W_k[w_k, w_{k+1}, t, s] = <t| O |s>, boundary rows folded in
    so that w_0 = w_N = 1.
  * classifier site k: [D_k, d, D_{k+1}], except the label site
    [D_c, d, n_labels, D_{c+1}]; pixels [B, N] in [0, 1).

The workloads stand in for the paper's use cases (section IV): random MPS for
the physics chain, and uniform-random 28x28 greyscale images in place of
MNIST, which is not available here.
"""
from __future__ import annotations

import numpy as np

# --------------------------------------------------------------------------
# MPS
# --------------------------------------------------------------------------


def bond_dims(n_sites: int, d: int, chi: int) -> list[int]:
    """D_k = min(chi, d^k, d^(N-k)) for k = 0..N (open boundaries)."""
    out = []
    for k in range(n_sites + 1):
        e = min(k, n_sites - k)
        v = 1
        for _ in range(e):
            v *= d
            if v >= chi:
                break
        out.append(min(chi, v))
    return out


def random_mps(n_sites: int, d: int, chi: int, seed, dims=None) -> list[np.ndarray]:
    """Entries i.i.d. N(0,1)/sqrt(chi*d), using the nominal chi for the scale."""
    rng = np.random.default_rng(seed)
    dims = bond_dims(n_sites, d, chi) if dims is None else dims
    scale = 1.0 / np.sqrt(chi * d)
    return [rng.standard_normal((dims[k], d, dims[k + 1])) * scale for k in range(n_sites)]


def correlated_mps_pair(n_sites: int, d: int, chi: int, seed, noise: float = 0.1):
    """psi random; phi = psi + noise * G with G an independent copy (same dims)."""
    rng = np.random.default_rng(seed)
    dims = bond_dims(n_sites, d, chi)
    scale = 1.0 / np.sqrt(chi * d)
    psi = [rng.standard_normal((dims[k], d, dims[k + 1])) * scale for k in range(n_sites)]
    g = [rng.standard_normal((dims[k], d, dims[k + 1])) * scale for k in range(n_sites)]
    phi = [p + noise * q for p, q in zip(psi, g)]
    return psi, phi


def uneven_chain_shapes(n_chains: int = 512, seed: int = 403, n_range=(8, 256), chi_range=(8, 512)):
    """Per-chain (N_i, chi_i) with N ~ U{n_range}, chi ~ U{chi_range} (inclusive)."""
    rng = np.random.default_rng(seed)
    ns = rng.integers(n_range[0], n_range[1] + 1, size=n_chains)
    chis = rng.integers(chi_range[0], chi_range[1] + 1, size=n_chains)
    return [(int(a), int(b)) for a, b in zip(ns, chis)]


def uneven_chain(i: int, n_sites: int, chi: int, seed: int = 403, d: int = 2):
    """Chain i of the uneven batch: a correlated pair seeded by [seed, i].

    Drawn and combined in float32 (psi = N(0,1) * scale, phi = psi + 0.1 G,
    each step one IEEE float32 operation), so that the full 512-chain
    workload (about 84 GB) can be streamed to the device chain by chain in a
    few tens of seconds while any single chain is reproduced bit for bit.
    Returns two lists of float32 arrays [D_k, d, D_{k+1}]."""
    rng = np.random.default_rng([seed, i])
    dims = bond_dims(n_sites, d, chi)
    scale = np.float32(1.0 / np.sqrt(chi * d))
    noise = np.float32(0.1)
    psi = [rng.standard_normal((dims[k], d, dims[k + 1]), dtype=np.float32) * scale for k in range(n_sites)]
    phi = [p + noise * (rng.standard_normal(p.shape, dtype=np.float32) * scale) for p in psi]
    return psi, phi


def uneven_chain_flat(i: int, n_sites: int, chi: int, seed: int = 403, d: int = 2):
    """uneven_chain(i, ...) packed as one float32 buffer: psi's sites then
    phi's, each site row-major.  Returns (buffer, shapes)."""
    psi, phi = uneven_chain(i, n_sites, chi, seed, d)
    shapes = [x.shape for x in psi]
    return np.concatenate([x.ravel() for x in psi + phi]), shapes


# --------------------------------------------------------------------------
# Spin-chain operators as MPOs (model constants, no contraction)
# --------------------------------------------------------------------------

_I2 = np.eye(2)
_X = np.array([[0.0, 1.0], [1.0, 0.0]])
_Z = np.array([[1.0, 0.0], [0.0, -1.0]])
_SP = np.array([[0.0, 1.0], [0.0, 0.0]])   # S^+ = |up><down| with |up> = basis 0
_SM = _SP.T.copy()
_SZ = 0.5 * _Z


def _fold_boundaries(bulk: np.ndarray, n_sites: int, first_row: int, last_col: int):
    w = bulk.shape[0]
    out = []
    for k in range(n_sites):
        t = bulk
        if k == 0:
            t = t[first_row:first_row + 1]
        if k == n_sites - 1:
            t = t[:, last_col:last_col + 1]
        out.append(np.ascontiguousarray(t))
    assert all(x.shape[0] in (1, w) for x in out)
    return out


def tfim_mpo(n_sites: int, J: float = 1.0, g: float = 1.0) -> list[np.ndarray]:
    """H = -J sum Z_i Z_{i+1} - g sum X_i as a bond-3 MPO W[u, v, t, s]."""
    w = np.zeros((3, 3, 2, 2))
    w[0, 0] = _I2
    w[0, 1] = -J * _Z
    w[0, 2] = -g * _X
    w[1, 2] = _Z
    w[2, 2] = _I2
    return _fold_boundaries(w, n_sites, 0, 2)


def xxz_mpo(n_sites: int, delta: float = 0.5) -> list[np.ndarray]:
    """H = sum (Sx Sx + Sy Sy + delta Sz Sz) (spin 1/2) as a bond-5 MPO."""
    w = np.zeros((5, 5, 2, 2))
    w[0, 0] = _I2
    w[0, 1] = 0.5 * _SP
    w[0, 2] = 0.5 * _SM
    w[0, 3] = delta * _SZ
    w[1, 4] = _SM
    w[2, 4] = _SP
    w[3, 4] = _SZ
    w[4, 4] = _I2
    return _fold_boundaries(w, n_sites, 0, 4)


# --------------------------------------------------------------------------
# Classifier (section IV.A workload, synthetic)
# --------------------------------------------------------------------------


def classifier_sites(n_sites: int, chi: int, n_labels: int, label_site: int, seed, d: int = 2):
    """Uniform bond chi with dimension-1 ends; entries N(0,1)/sqrt(chi)."""
    rng = np.random.default_rng(seed)
    dims = [1] + [chi] * (n_sites - 1) + [1]
    scale = 1.0 / np.sqrt(chi)
    sites = []
    for k in range(n_sites):
        if k == label_site:
            shape = (dims[k], d, n_labels, dims[k + 1])
        else:
            shape = (dims[k], d, dims[k + 1])
        sites.append(rng.standard_normal(shape) * scale)
    return sites


def images(batch: int, n_pixels: int, seed) -> np.ndarray:
    """Pixels ~ U[0, 1), row-major [B, N]."""
    return np.random.default_rng(seed).random((batch, n_pixels))


def labels(batch: int, n_labels: int, seed) -> np.ndarray:
    return np.random.default_rng(seed).integers(0, n_labels, size=batch).astype(np.int64)


def random_directions(shapes, seed) -> list[np.ndarray]:
    rng = np.random.default_rng(seed)
    return [rng.standard_normal(s) for s in shapes]


def random_mps_complex(n_sites: int, d: int, chi: int, seed, dims=None) -> list[np.ndarray]:
    """Complex sites: real and imaginary parts i.i.d. N(0,1)/sqrt(2 chi d)."""
    rng = np.random.default_rng(seed)
    dims = bond_dims(n_sites, d, chi) if dims is None else dims
    scale = 1.0 / np.sqrt(2 * chi * d)
    return [(rng.standard_normal((dims[k], d, dims[k + 1])) + 1j * rng.standard_normal((dims[k], d, dims[k + 1])))
            * scale for k in range(n_sites)]
