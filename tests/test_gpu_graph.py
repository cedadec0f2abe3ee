"""Library call sequences recorded as HIP graphs (Graph) and replayed.

Every replay is checked against the eager result; between replays the
outputs are poisoned with NaN and unrelated eager work runs, with
synchronisations, so a replay that reused stale values or skipped a step
would show.  The kernels are deterministic, so replays must match exactly.
"""
import numpy as np
import pytest
import torch

import paper_1905_01330_amd as tn
from paper_1905_01330_amd import inputs

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


def eager_noise():
    x = torch.randn(1 << 20, device=DEV)
    y = (x * 2.0).cumsum(0)
    torch.cuda.synchronize()
    return float(y[-1])


def replay_and_check(graph, outputs, expected, reps=3):
    for _ in range(reps):
        for o in outputs:
            o.fill_(float("nan"))
        eager_noise()
        graph.replay()
        torch.cuda.synchronize()
        for o, e in zip(outputs, expected):
            assert torch.equal(o, e)


def test_env_sweep_graph():
    n, chi = 14, 32
    psi = [torch.tensor(x, dtype=torch.float64, device=DEV) for x in inputs.random_mps(n, 2, chi, 11)]
    tn.mps_left_canonicalize(psi)
    psi = [s.float().contiguous() for s in psi]
    mpo = [torch.tensor(w, dtype=torch.float32, device=DEV) for w in inputs.tfim_mpo(n, 1.0, 1.0)]
    sweep = tn.EnvSweep(psi, mpo, left=True, right=True, store=True, prec="split_bf16")
    sweep.run()
    torch.cuda.synchronize()
    expected = [sweep.energy.clone()] + [t.clone() for t in sweep.L] + [t.clone() for t in sweep.R]
    g = tn.Graph(sweep.run)
    replay_and_check(g, [sweep.energy] + sweep.L + sweep.R, expected)


def test_batched_inner_graph():
    shapes = [(9, 16), (13, 40), (20, 8), (11, 64), (16, 24)]
    chains = []
    for i, (n, chi) in enumerate(shapes):
        p = inputs.random_mps(n, 2, chi, 500 + i)
        q = inputs.random_mps(n, 2, chi, 600 + i)
        q = [a + 0.1 * b for a, b in zip(p, q)]
        chains.append(([torch.tensor(x, dtype=torch.float32, device=DEV) for x in p],
                       [torch.tensor(x, dtype=torch.float32, device=DEV) for x in q]))
    b = tn.BatchedInner(chains, prec="fp32")
    expected = [b.run().clone()]
    torch.cuda.synchronize()
    g = tn.Graph(b.run)
    replay_and_check(g, [b.out2], expected)


def test_classifier_forward_backward_graph():
    n, chi, L, c, B = 30, 16, 10, 14, 40
    sites = [torch.tensor(s, dtype=torch.float32, device=DEV) for s in inputs.classifier_sites(n, chi, L, c, 3)]
    pix = torch.tensor(inputs.images(B, n, 4), dtype=torch.float32, device=DEV)
    lab = torch.tensor(inputs.labels(B, L, 5), device=DEV)
    model = tn.MPSClassifier(n, c, L, chi, B, ckpt_every=7, prec="split_bf16")
    logits = torch.empty((B, L), device=DEV)
    dlog = torch.empty((B, L), device=DEV)
    dsites = [torch.empty_like(s) for s in sites]

    def step():
        model.forward(sites, pix, logits)
        _, d = tn.softmax_xent(logits, lab)
        dlog.copy_(d)
        model.backward(sites, pix, dlog, dsites)

    step()
    torch.cuda.synchronize()
    expected = [logits.clone()] + [d.clone() for d in dsites]
    g = tn.Graph(step)
    replay_and_check(g, [logits] + dsites, expected)


def test_contraction_graph_with_permuted_output():
    rng = np.random.default_rng(7)
    a = torch.tensor(rng.standard_normal((48, 5, 40)), dtype=torch.float32, device=DEV)
    b = torch.tensor(rng.standard_normal((40, 2, 56)), dtype=torch.float32, device=DEV)
    base = torch.empty((56, 2, 5, 48), device=DEV)
    out = base.permute(3, 2, 1, 0)   # [48, 5, 2, 56] view of a transposed buffer
    tn.contract_between(a, b, [2], [0], out=out, prec="split_bf16")
    torch.cuda.synchronize()
    expected = [base.clone()]
    g = tn.Graph(lambda: tn.contract_between(a, b, [2], [0], out=out, prec="split_bf16"))
    replay_and_check(g, [base], expected)


def test_two_sided_inner_graph():
    """A single inner product of 4+ sites forks its right half onto the
    library's side stream and joins it back: both halves must be recorded."""
    n, chi = 12, 48
    psi = [torch.tensor(x, dtype=torch.float32, device=DEV) for x in inputs.random_mps(n, 2, chi, 21)]
    phi = [torch.tensor(x, dtype=torch.float32, device=DEV) for x in inputs.random_mps(n, 2, chi, 22)]
    expected = [tn.mps_inner(psi, phi, prec="split_bf16").clone()]
    torch.cuda.synchronize()
    g = tn.Graph(lambda: tn.mps_inner(psi, phi, prec="split_bf16"))
    replay_and_check(g, [g.result], expected)
