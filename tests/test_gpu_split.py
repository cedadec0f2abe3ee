"""GPU parity of node splitting (section III.B "Node Splitting", Appendix A
"Saving Memory") against the FP64 oracle.

Singular vectors are fixed only up to sign (and rotations inside degenerate
subspaces), so the comparison uses what is unique: the singular values, the
dropped values, the rank chosen by the truncation rule, the products of the
factors and the projectors onto the kept subspace; the factors' own
properties (isometries, the even split of the square roots) are checked on
the GPU's output directly.  FP64 nodes: 1e-12 relative to the largest
singular value; FP32 nodes (decomposed in FP64, written as FP32): 1e-6."""
import numpy as np
import pytest
import torch

import oracle
import paper_1905_01330_amd as tn
from helpers import random_orthogonal

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


def known_spectrum(m, n, s, seed):
    rng = np.random.default_rng(seed)
    r = len(s)
    return (random_orthogonal(m, rng)[:, :r] * np.asarray(s)[None, :]) @ random_orthogonal(n, rng)[:, :r].T


def host(t):
    return t.cpu().double().numpy()


def check_full(a, left_axes, right_axes, dtype, max_sv=None, max_err=None):
    """Decompose on the GPU in both forms and compare with the oracle; returns k."""
    tol = 1e-12 if dtype == torch.float64 else 1e-6
    ga = torch.tensor(a, dtype=dtype, device=DEV)
    ah = host(ga)                                     # the node as the GPU sees it
    perm = list(left_axes) + list(right_axes)
    ap = np.transpose(ah, perm)
    nl = len(left_axes)
    u_r, s_r, vt_r, tr_r = oracle.split_node_full_svd(ap, nl, max_sv, max_err)
    smax = s_r[0, 0]
    u, s, vt, tr = tn.split_node_full_svd(ga, left_axes, right_axes, max_sv, max_err)
    torch.cuda.synchronize()
    k = s.shape[0]
    assert k == s_r.shape[0], (k, s_r.shape[0])
    assert tuple(u.shape) == u_r.shape and tuple(vt.shape) == vt_r.shape and tuple(tr.shape) == tr_r.shape
    np.testing.assert_allclose(np.diag(host(s)), np.diag(s_r), atol=tol * smax, rtol=0)
    assert np.allclose(host(s) - np.diag(np.diag(host(s))), 0.0)
    np.testing.assert_allclose(host(tr), tr_r, atol=tol * smax, rtol=0)
    um, vm = host(u).reshape(-1, k), host(vt).reshape(k, -1)
    nz = np.diag(s_r) > 1e-10 * smax                   # vectors of nonzero values are orthonormal
    np.testing.assert_allclose((um.T @ um)[np.ix_(nz, nz)], np.eye(int(nz.sum())), atol=10 * tol)
    np.testing.assert_allclose((vm @ vm.T)[np.ix_(nz, nz)], np.eye(int(nz.sum())), atol=10 * tol)
    # the truncated product equals the oracle's (unique when the cut is not inside a degenerate cluster)
    mat = ap.reshape(um.shape[0], vm.shape[1])
    prod = (um * np.diag(host(s))) @ vm
    prod_r = (u_r.reshape(-1, k) * np.diag(s_r)) @ vt_r.reshape(k, -1)
    assert np.linalg.norm(prod - prod_r) <= 10 * tol * np.linalg.norm(mat)
    # split_node form: the square roots split evenly and the factors multiply back
    left, right, tr2 = tn.split_node(ga, left_axes, right_axes, max_sv, max_err)
    torch.cuda.synchronize()
    lm, rm = host(left).reshape(-1, k), host(right).reshape(k, -1)
    np.testing.assert_allclose(np.linalg.norm(lm, axis=0) ** 2, np.diag(s_r), atol=10 * tol * smax, rtol=0)
    np.testing.assert_allclose(np.linalg.norm(rm, axis=1) ** 2, np.diag(s_r), atol=10 * tol * smax, rtol=0)
    assert np.linalg.norm(lm @ rm - prod_r) <= 10 * tol * np.linalg.norm(mat)
    np.testing.assert_allclose(host(tr2), tr_r, atol=tol * smax, rtol=0)
    return k


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_paper_shape_split(dtype):
    """(2, 3, 4, 5, 6) with the first three legs on the left: (2,3,4,24) and (24,5,6)."""
    a = np.random.default_rng(1).standard_normal((2, 3, 4, 5, 6))
    left, right, tr = tn.split_node(torch.tensor(a, dtype=dtype, device=DEV), [0, 1, 2], [3, 4])
    assert tuple(left.shape) == (2, 3, 4, 24) and tuple(right.shape) == (24, 5, 6) and tuple(tr.shape) == (0,)
    assert check_full(a, [0, 1, 2], [3, 4], dtype) == 24


def test_paper_truncation_1000_by_1000():
    """Appendix A: max_singular_values = 5 gives (1000, 5), (5, 1000), trun_err (995,);
    max_truncation_err = 0.1 drops values adding up to at most 0.1."""
    s = np.exp(-np.arange(1000) / 40.0)
    a = known_spectrum(1000, 1000, s, 7)
    ga = torch.tensor(a, device=DEV)
    left, right, tr = tn.split_node(ga, [0], [1], max_singular_values=5)
    assert tuple(left.shape) == (1000, 5) and tuple(right.shape) == (5, 1000) and tuple(tr.shape) == (995,)
    np.testing.assert_allclose(host(tr), s[5:], atol=1e-12, rtol=0)
    assert check_full(a, [0], [1], torch.float64, max_sv=5) == 5
    k = check_full(a, [0], [1], torch.float64, max_err=0.1)
    _, _, tr = tn.split_node(ga, [0], [1], max_truncation_err=0.1)
    assert float(tr.sum()) <= 0.1 and k == 1000 - tr.shape[0]


@pytest.mark.parametrize("shape,left,right", [
    ((37, 53), [0], [1]),                 # ragged, tall after transposition
    ((53, 37), [0], [1]),
    ((7, 3, 5, 11), [0, 1], [2, 3]),      # 21 x 55: the work matrix is A^T
    ((6, 9, 10), [2, 0], [1]),            # permuted legs
    ((130, 70), [0], [1]),                # several blocks, odd block count padded
])
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_shapes_and_layouts(shape, left, right, dtype):
    a = np.random.default_rng(sum(shape)).standard_normal(shape)
    check_full(a, left, right, dtype)
    check_full(a, left, right, dtype, max_sv=3)


def test_strided_input_view():
    a = np.random.default_rng(4).standard_normal((20, 31))
    big = torch.tensor(np.random.default_rng(5).standard_normal((40, 62)), device=DEV)
    big[::2, ::2] = torch.tensor(a, device=DEV)
    view = big[::2, ::2]
    u, s, vt, _ = tn.split_node_full_svd(view, [0], [1])
    _, s_r, _, _ = oracle.split_node_full_svd(a, 1)
    np.testing.assert_allclose(np.diag(host(s)), np.diag(s_r), atol=1e-12 * s_r[0, 0])


def test_rank_deficient_and_degenerate():
    rng = np.random.default_rng(6)
    x, y = rng.standard_normal(40), rng.standard_normal(25)
    a = np.multiply.outer(x, y)
    u, s, vt, tr = tn.split_node_full_svd(torch.tensor(a, device=DEV), [0], [1])
    sv = np.diag(host(s))
    assert abs(sv[0] - np.linalg.norm(x) * np.linalg.norm(y)) <= 1e-12 * sv[0]
    assert np.all(sv[1:] <= 1e-12 * sv[0])
    left, right, tr = tn.split_node(torch.tensor(a, device=DEV), [0], [1], max_truncation_err=1e-9)
    assert left.shape[1] == 1 and tr.shape[0] == 24 and float(tr.sum()) <= 1e-9
    np.testing.assert_allclose(host(left) @ host(right), a, atol=1e-12 * np.abs(a).max())
    # a spectrum with repeated values: the values and the product are unique
    sdeg = np.array([5.0, 5.0, 5.0, 2.0, 2.0, 1.0, 0.5, 0.5])
    check_full(known_spectrum(30, 20, sdeg, 8), [0], [1], torch.float64, max_sv=5)


def decompose_sweeps(ga, n_left):
    """Jacobi sweeps the decomposition of ga (left legs first) takes, through the C-ABI."""
    import ctypes as C
    from paper_1905_01330_amd import _lib as L
    da = L.tensor_desc(ga)
    nbytes = C.c_size_t(0)
    L.check(L.lib().tn_split_node_workspace(C.byref(da), n_left, C.byref(nbytes)))
    ws = torch.empty(nbytes.value, dtype=torch.uint8, device=DEV)
    k, sweeps = C.c_int32(0), C.c_int32(0)
    L.check(L.lib().tn_split_node_decompose(C.byref(da), n_left, -1, -1.0, C.byref(k), C.byref(sweeps),
                                            C.c_void_p(ws.data_ptr()), nbytes.value, L.stream_ptr()))
    return k.value, sweeps.value


def test_preconditioned_sweeps_on_a_graded_spectrum():
    """The sweeps run on R^T of a Householder QR: on the graded 1000 x 1000 node
    (e^(-i/40)) they converge in far fewer sweeps than the 41 the node itself
    takes, and the values stay those of the oracle."""
    s = np.exp(-np.arange(1000) / 40.0)
    ga = torch.tensor(known_spectrum(1000, 1000, s, 7), device=DEV)
    k, sweeps = decompose_sweeps(ga, 1)
    print("graded 1000 x 1000: sweeps", sweeps)
    assert k == 1000 and sweeps <= 20


def test_preconditioned_rank_deficient():
    """Rank 3 in a 120 x 64 node and an all-zero 40 x 36 node (both wide enough
    for the QR-preconditioned sweeps): zero values, zero vectors for them, no NaN."""
    a = known_spectrum(120, 64, [3.0, 2.0, 1.0], 9)
    check_full(a, [0], [1], torch.float64)
    left, right, tr = tn.split_node(torch.tensor(a, device=DEV), [0], [1], max_truncation_err=1e-9)
    assert left.shape[1] == 3 and tr.shape[0] == 61
    np.testing.assert_allclose(host(left) @ host(right), a, atol=1e-12 * 3.0)
    z = torch.zeros((40, 36), dtype=torch.float64, device=DEV)
    u, sv, vt, tr = tn.split_node_full_svd(z, [0], [1])
    for t in (u, sv, vt, tr):
        assert torch.isfinite(t).all()
    assert sv.numel() == 0 or float(sv.abs().max()) == 0.0


@pytest.mark.parametrize("shape", [(2100, 40), (40, 2100), (2048, 48)])
def test_long_side_at_and_past_the_qr_rows(shape):
    """A long side of 2048 rows (the most the blocked QR takes) and past it,
    where the sweeps run on the node itself."""
    a = np.random.default_rng(shape[0]).standard_normal(shape)
    check_full(a, [0], [1], torch.float64)


def test_errors_before_launch():
    a = torch.zeros((4, 5), device=DEV, dtype=torch.float64)
    with pytest.raises(ValueError):
        tn.split_node(a, [0], [0])
