"""GPU parity of the MPS classifier (section IV.A): scores, cross-entropy,
and the gradient with respect to every site tensor, against the FP64 oracle.

Gates: scores within 1e-5 relative per sample (FP64 chain products, FP32
storage of the vectors between kernel runs and of the site tensors), loss
within 1e-5 relative, gradients within 1e-4 relative (Frobenius, over all
sites and per site) of the FP64 oracle gradient.
"""
import math

import numpy as np
import pytest
import torch

import oracle
import paper_1905_01330_amd as tn
from paper_1905_01330_amd import inputs

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


def setup(n, chi, L, c, B, seed, scale=1.0):
    sites = [s * scale for s in inputs.classifier_sites(n, chi, L, c, seed)]
    sites = [s.astype(np.float32).astype(np.float64) for s in sites]
    pix = inputs.images(B, n, seed + 1).astype(np.float32).astype(np.float64)
    lab = inputs.labels(B, L, seed + 2)
    g_sites = [torch.tensor(s, dtype=torch.float32, device=DEV) for s in sites]
    g_pix = torch.tensor(pix, dtype=torch.float32, device=DEV)
    g_lab = torch.tensor(lab, dtype=torch.int64, device=DEV)
    return sites, pix, lab, g_sites, g_pix, g_lab


def rel_rows(got, ref):
    return np.max(np.linalg.norm(got - ref, axis=1) / np.linalg.norm(ref, axis=1))


@pytest.mark.parametrize("prec", ["fp32", "split_bf16"])
@pytest.mark.parametrize("shape", [(12, 8, 3, 5, 20, 4), (40, 32, 10, 19, 37, 7), (30, 64, 10, 14, 64, 28)])
def test_forward_and_gradient_vs_oracle(shape, prec):
    n, chi, L, c, B, E = shape
    sites, pix, lab, gs, gp, gl = setup(n, chi, L, c, B, 11 + n)
    model = tn.MPSClassifier(n, c, L, chi, B, ckpt_every=E, prec=prec)
    logits = model.forward(gs, gp)
    torch.cuda.synchronize()
    ref = oracle.classifier_forward(sites, c, pix)
    assert rel_rows(logits.cpu().double().numpy(), ref) <= 1e-5
    loss, dlog = tn.softmax_xent(logits, gl)
    loss_ref, grads_ref = oracle.classifier_loss_and_grad(sites, c, pix, lab)
    assert abs(float(loss.cpu()) - loss_ref) <= 1e-5 * abs(loss_ref)
    dsites = model.backward(gs, gp, dlog)
    torch.cuda.synchronize()
    num = sum(float(np.sum((d.cpu().double().numpy() - r) ** 2)) for d, r in zip(dsites, grads_ref))
    den = sum(float(np.sum(r ** 2)) for r in grads_ref)
    assert math.sqrt(num / den) <= 1e-4, math.sqrt(num / den)
    for k in (0, c - 1, c, c + 1, n - 1):
        d, r = dsites[k].cpu().double().numpy(), grads_ref[k]
        assert np.linalg.norm(d - r) <= 1e-4 * np.linalg.norm(r) + 1e-30, k


def test_forward_without_checkpoint_buffer_matches():
    n, chi, L, c, B = 70, 16, 4, 33, 50
    sites, pix, lab, gs, gp, gl = setup(n, chi, L, c, B, 5)
    model = tn.MPSClassifier(n, c, L, chi, B, ckpt_every=8)
    a = model.forward(gs, gp).cpu().numpy()
    from paper_1905_01330_amd import _lib as Lb
    import ctypes as C
    out = torch.empty((B, L), device=DEV)
    ds, dp, dl = Lb.tensor_array(gs), Lb.tensor_desc(gp), Lb.tensor_desc(out)
    Lb.check(Lb.lib().tn_mps_classifier_forward(n, c, L, ds, C.byref(dp), C.byref(dl), None, 8,
                                                C.c_void_p(model.ws.data_ptr()), model.nbytes, 0, Lb.stream_ptr()))
    torch.cuda.synchronize()
    # both round the FP64 running vector to FP32 between kernel runs, at
    # different sites (checkpoints versus 64-site runs): agree per sample
    assert rel_rows(out.cpu().double().numpy(), a.astype(np.float64)) <= 1e-5


def test_long_chain_rescaling():
    """784 sites; left sites scaled by 1.5 and right sites by 1/1.5: the left
    vectors grow like 1.5^392 ~ 1e69 and the right ones shrink alike, so raw
    FP32 chains would overflow and underflow while the scores stay moderate.
    The per-sample power-of-two exponents keep them exact."""
    n, chi, L, c, B = 784, 16, 10, 392, 16
    sites, pix, lab, gs, gp, gl = setup(n, chi, L, c, B, 7)
    sites = [s * (1.5 if k < c else (1 / 1.5 if k > c else 1.0)) for k, s in enumerate(sites)]
    sites = [s.astype(np.float32).astype(np.float64) for s in sites]
    gs = [torch.tensor(s, dtype=torch.float32, device=DEV) for s in sites]
    ref = oracle.classifier_forward(sites, c, pix)
    assert np.all(np.isfinite(ref)) and np.max(np.abs(ref)) < 1e30
    model = tn.MPSClassifier(n, c, L, chi, B)
    got = model.forward(gs, gp).cpu().double().numpy()
    assert rel_rows(got, ref) <= 5e-5


def test_autograd_function_and_gpu_finite_difference():
    n, chi, L, c, B = 20, 8, 4, 9, 24
    sites, pix, lab, gs, gp, gl = setup(n, chi, L, c, B, 3, scale=1.2)
    model = tn.MPSClassifier(n, c, L, chi, B, ckpt_every=5)
    params = [s.clone().requires_grad_(True) for s in gs]
    logits = tn.ClassifierFunction.apply(model, gp, *params)
    grads = torch.autograd.grad(logits, params, grad_outputs=tn.softmax_xent(logits.detach(), gl)[1])
    _, gref = oracle.classifier_loss_and_grad(sites, c, pix, lab)
    for g, r in zip(grads, gref):
        assert np.linalg.norm(g.cpu().double().numpy() - r) <= 1e-4 * np.linalg.norm(r) + 1e-30
    # central difference of the GPU loss along one site's direction (FP32 loss: loose gate)
    k = 4
    d = torch.tensor(inputs.random_directions([sites[k].shape], 9)[0], dtype=torch.float32, device=DEV)
    d *= torch.linalg.norm(gs[k]) / torch.linalg.norm(d)
    eps = 1e-2

    def loss_at(t):
        s2 = list(gs)
        s2[k] = gs[k] + t * d
        return float(tn.softmax_xent(model.forward(s2, gp), gl)[0].cpu())

    fd = (loss_at(eps) - loss_at(-eps)) / (2 * eps)
    an = float((grads[k] * d).sum())
    assert abs(fd - an) <= 2e-3 * abs(an) + 1e-6


def test_softmax_xent_matches_oracle():
    rng = np.random.default_rng(1)
    f = rng.standard_normal((300, 10)).astype(np.float32) * 3
    y = rng.integers(0, 10, 300)
    loss, d = tn.softmax_xent(torch.tensor(f, device=DEV), torch.tensor(y, device=DEV))
    f64 = f.astype(np.float64)
    m = f64.max(1, keepdims=True)
    p = np.exp(f64 - m)
    p /= p.sum(1, keepdims=True)
    ref = float(np.mean(-np.log(p[np.arange(300), y])))
    assert abs(float(loss.cpu()) - ref) < 1e-12 * abs(ref) + 1e-12
    g = p.copy()
    g[np.arange(300), y] -= 1
    g /= 300
    np.testing.assert_allclose(d.cpu().double().numpy(), g, rtol=1e-6, atol=1e-9)
