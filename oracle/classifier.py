"""Oracle: MPS classifier scores, cross-entropy loss and gradient (FP64).

Test infrastructure only (see the package docstring).

Section IV.A: each pixel p is encoded by the local feature map
Phi(p) = (cos(pi p/2), sin(pi p/2)); the image is the tensor product of
those vectors and a label's score is the inner product of that product
state with the MPS.  Here a single MPS carries all labels through a label
leg on the centre site c:
  f[b, l] = sum v_c[b, a] Phi_s(x_{b,c}) A_c[a, s, l, z] u_{c+1}[b, z]
with v_0 = 1, v_{k+1}[b, z] = sum_{a,s} v_k[b, a] Phi_s(x_{b,k}) A_k[a, s, z]
and  u_N = 1, u_k[b, a]     = sum_{s,z} A_k[a, s, z] Phi_s(x_{b,k}) u_{k+1}[b, z].
The loss is the batch-mean softmax cross-entropy; the gradient is taken by
the chain rule through these recursions, with every v_k and u_k stored.
"""
from __future__ import annotations

import numpy as np

from .contract import feature_map, tensordot


def _left_vectors(sites, phi, label_site):
    b = phi.shape[0]
    v = [np.ones((b, 1))]
    for k in range(label_site):
        x = v[-1][:, :, None] * phi[:, k, None, :]            # [b, a, s]
        v.append(tensordot(x, sites[k], [1, 2], [0, 1]))        # [b, z]
    return v  # v[k] for k = 0..c


def _right_vectors(sites, phi, label_site):
    n = len(sites)
    b = phi.shape[0]
    u = {n: np.ones((b, 1))}
    for k in range(n - 1, label_site, -1):
        y = tensordot(u[k + 1], sites[k], [1], [2])             # [b, a, s]
        u[k] = np.sum(y * phi[:, k, None, :], axis=2)           # [b, a]
    return u  # u[k] for k = c+1..N


def classifier_forward(sites, label_site, pixels):
    """Scores f[b, l] (FP64), exactly as the section IV.A inner product."""
    phi = feature_map(pixels)                                   # [B, N, 2]
    v = _left_vectors(sites, phi, label_site)
    u = _right_vectors(sites, phi, label_site)
    x = v[label_site][:, :, None] * phi[:, label_site, None, :]  # [b, a, s]
    t = tensordot(x, sites[label_site], [1, 2], [0, 1])         # [b, l, z]
    return np.einsum("blz,bz->bl", t, u[label_site + 1])


def classifier_loss(sites, label_site, pixels, labels):
    f = classifier_forward(sites, label_site, pixels)
    m = np.max(f, axis=1, keepdims=True)
    lse = m[:, 0] + np.log(np.sum(np.exp(f - m), axis=1))
    return float(np.mean(lse - f[np.arange(f.shape[0]), labels]))


def classifier_loss_and_grad(sites, label_site, pixels, labels):
    """Loss and d loss / d A_k for every site (list with the sites' shapes)."""
    n = len(sites)
    c = label_site
    phi = feature_map(pixels)
    bsz = phi.shape[0]
    v = _left_vectors(sites, phi, c)
    u = _right_vectors(sites, phi, c)
    xc = v[c][:, :, None] * phi[:, c, None, :]                  # [b, a, s]
    t = tensordot(xc, sites[c], [1, 2], [0, 1])                 # [b, l, z]
    f = np.einsum("blz,bz->bl", t, u[c + 1])
    m = np.max(f, axis=1, keepdims=True)
    e = np.exp(f - m)
    z = np.sum(e, axis=1, keepdims=True)
    p = e / z
    lse = m[:, 0] + np.log(z[:, 0])
    loss = float(np.mean(lse - f[np.arange(bsz), labels]))
    g = p.copy()
    g[np.arange(bsz), labels] -= 1.0
    g /= bsz                                                    # dL/df [b, l]

    grads = [None] * n
    # label site: dA_c[a, s, l, z] = sum_b g[b, l] xc[b, a, s] u_{c+1}[b, z]
    gu = g[:, :, None] * u[c + 1][:, None, :]                   # [b, l, z]
    grads[c] = tensordot(xc, gu, [0], [0])                      # [a, s, l, z]
    # adjoint of v_c: abar[b, a] = sum_{s,l,z} phi_s A_c[a, s, l, z] g[b,l] u[b,z]
    y = tensordot(gu, sites[c], [1, 2], [2, 3])                 # [b, a, s]
    abar = np.sum(y * phi[:, c, None, :], axis=2)               # [b, a]
    for k in range(c - 1, -1, -1):
        xk = v[k][:, :, None] * phi[:, k, None, :]              # [b, a, s]
        grads[k] = tensordot(xk, abar, [0], [0])                # [a, s, z]
        yk = tensordot(abar, sites[k], [1], [2])                # [b, a, s]
        abar = np.sum(yk * phi[:, k, None, :], axis=2)
    # adjoint of u_{c+1}: ubar[b, z] = sum_{l,a,s} g[b,l] xc[b,a,s] A_c[a,s,l,z]
    ubar = np.einsum("blz,bl->bz", t, g)
    for k in range(c + 1, n):
        grads[k] = tensordot(ubar[:, :, None] * phi[:, k, None, :], u[k + 1], [0], [0])  # [a, s, z]
        xk = ubar[:, :, None] * phi[:, k, None, :]
        ubar = tensordot(xk, sites[k], [1, 2], [0, 1])          # [b, z]
    return loss, grads
