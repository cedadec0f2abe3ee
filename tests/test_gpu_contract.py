"""GPU parity of the pairwise contraction, trace, outer product and ncon
network entry points against the FP64 oracle.

Tolerances (relative Frobenius error against the oracle run on the same
FP32-rounded inputs): FP32 1e-5 and SPLIT_BF16 1e-6 (the stated accuracy
targets), SPLIT_BF16_3P 1e-4 and plain BF16 2e-2 (reported precisions: the
bounds only catch gross errors).  Element-wise, every output must also be
within tol * (|A| |B|)_ij, the scale of the sum that produced it.
"""
import itertools
import json
import os

import numpy as np
import pytest
import torch

import oracle
import paper_1905_01330_amd as tn

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")
TOL = {"fp32": 1e-5, "split_bf16": 1e-6, "split_bf16_3p": 1e-4, "bf16": 2e-2}
PRECS = list(TOL)
GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_examples.json")))


def f32(x):
    return np.asarray(x, dtype=np.float32)


def gpu(x):
    return torch.tensor(np.asarray(x, dtype=np.float32), device=DEV)


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().double().numpy()


def check(got, ref, scale, tol, what=""):
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    assert got.shape == ref.shape, (got.shape, ref.shape)
    den = np.linalg.norm(ref.ravel())
    rel = np.linalg.norm((got - ref).ravel()) / (den if den > 0 else 1.0)
    assert rel <= tol, f"{what}: relative error {rel:.3e} > {tol:.1e}"
    bound = tol * 4 * scale + 1e-30
    bad = np.abs(got - ref) > bound
    assert not bad.any(), f"{what}: {bad.sum()} elements outside the element-wise bound"
    return rel


def abs_scale(a, b, pa, pb):
    return oracle.tensordot(np.abs(a), np.abs(b), pa, pb)


# ---------------------------------------------------------------------------
# the paper's examples


def test_paper_examples_on_gpu():
    g = GOLDEN["ones_dot"]
    c = tn.contract_between(gpu(g["a"]), gpu(g["b"]), [0], [0])
    assert float(host(c)) == g["value"]
    c = tn.contract_network([gpu(g["a"]), gpu(g["b"])], [[0], [0]])
    assert float(host(c)) == g["value"]
    g = GOLDEN["outer_shape"]
    rng = np.random.default_rng(1)
    a, b = f32(rng.standard_normal(g["shape_a"])), f32(rng.standard_normal(g["shape_b"]))
    c = tn.outer_product(gpu(a), gpu(b))
    assert list(c.shape) == g["shape_out"]
    np.testing.assert_array_equal(host(c), oracle.outer_product(a, b).astype(np.float32))
    g = GOLDEN["ncon_matmul"]
    a, b = f32(rng.standard_normal((2, 2))), f32(rng.standard_normal((2, 2)))
    c = tn.contract_network([gpu(a), gpu(b)], g["labels"])
    assert np.linalg.norm(host(c) - a.astype(np.float64) @ b.astype(np.float64)) < 1e-6
    c = tn.contract_network([gpu(np.eye(2)), gpu(np.eye(2))], [[0, 1], [0, 1]])
    assert float(host(c)) == 2.0
    h = np.array([[1.0, 1.0], [1.0, -1.0]]) / np.sqrt(2.0)
    out = tn.contract_network([gpu([1.0, 0.0])] + [gpu(h)] * 5, [[0]] + [[i + 1, i] for i in range(4)] + [[-1, 4]])
    np.testing.assert_allclose(host(out), [2 ** -0.5, 2 ** -0.5], rtol=1e-6)


# ---------------------------------------------------------------------------
# fuzzed pairwise contractions


def random_case(rng, max_dim=9, big=False):
    ra = int(rng.integers(1, 6))
    rb = int(rng.integers(1, 6))
    npairs = int(rng.integers(1, min(ra, rb) + 1))
    pa = [int(x) for x in rng.permutation(ra)[:npairs]]
    pb = [int(x) for x in rng.permutation(rb)[:npairs]]
    hi = 80 if big else max_dim
    sa = [int(rng.integers(1, hi)) for _ in range(ra)]
    sb = [int(rng.integers(1, hi)) for _ in range(rb)]
    for i, j in zip(pa, pb):
        sb[j] = sa[i]
    # keep sizes moderate
    while np.prod(sa) > 400_000:
        k = int(np.argmax(sa))
        sa[k] = max(1, sa[k] // 2)
        for i, j in zip(pa, pb):
            sb[j] = sa[i]
    while np.prod(sb) > 400_000:
        k = int(np.argmax(sb))
        sb[k] = max(1, sb[k] // 2)
        for i, j in zip(pa, pb):
            sa[i] = sb[j]
    return sa, sb, pa, pb


def permuted_input(x, rng):
    """The same tensor as a non-contiguous view: stored transposed, viewed back."""
    if x.ndim < 2:
        return gpu(x)
    perm = [int(p) for p in rng.permutation(x.ndim)]
    stored = gpu(np.transpose(x, perm).copy())
    inv = np.argsort(perm)
    return stored.permute(*[int(i) for i in inv])


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("seed", range(12))
def test_fuzz_contract_between(prec, seed):
    rng = np.random.default_rng(500 + seed)
    sa, sb, pa, pb = random_case(rng, big=seed % 3 == 0)
    a = f32(rng.standard_normal(sa))
    b = f32(rng.standard_normal(sb))
    ga = permuted_input(a, rng) if seed % 2 else gpu(a)
    gb = permuted_input(b, rng) if seed % 4 in (1, 2) else gpu(b)
    ref = oracle.tensordot(a, b, pa, pb)
    out_shape = ref.shape
    if len(out_shape) >= 2 and seed % 3 == 1:
        perm = [int(p) for p in rng.permutation(len(out_shape))]
        store = torch.empty([out_shape[p] for p in perm], device=DEV)
        out = store.permute(*[int(i) for i in np.argsort(perm)])
    else:
        out = torch.empty(out_shape, device=DEV)
    tn.contract_between(ga, gb, pa, pb, out=out, prec=prec)
    check(host(out), ref, abs_scale(a, b, pa, pb), TOL[prec], f"{sa}x{sb} pairs {pa}/{pb}")


@pytest.mark.parametrize("prec", PRECS)
def test_ragged_gemm_all_tiles(prec):
    rng = np.random.default_rng(7)
    a = f32(rng.standard_normal((197, 301)))
    b = f32(rng.standard_normal((301, 259)))
    ref = a.astype(np.float64) @ b.astype(np.float64)
    scale = np.abs(a).astype(np.float64) @ np.abs(b).astype(np.float64)
    try:
        for cfg in range(tn.tune_num_configs()):
            tn.tune_force_config(cfg)
            out = tn.contract_between(gpu(a), gpu(b), [1], [0], prec=prec)
            check(host(out), ref, scale, TOL[prec], f"tile config {cfg}")
    finally:
        tn.tune_force_config(-1)


@pytest.mark.parametrize("prec", PRECS)
def test_operands_of_odd_extent_all_tiles(prec):
    """A and B both read along k (unit stride) with K odd or small and rows
    that start anywhere (a one-float offset into the buffer, odd row
    pitches), then both row-contiguous with M and N odd: 16-byte loads at
    4-byte alignment and an element-by-element partial last block, on
    every tile configuration."""
    rng = np.random.default_rng(29)
    try:
        for M, K, N in [(197, 301, 163), (70, 3, 45), (33, 5, 64), (40, 130, 36)]:
            a = f32(rng.standard_normal((M, K)))
            b = f32(rng.standard_normal((K, N)))
            abuf = gpu(np.zeros(M * K + 1, dtype=np.float32))
            ga = abuf[1:].view(M, K)
            ga.copy_(gpu(a))
            bbuf = gpu(np.zeros(N * K + 1, dtype=np.float32))
            gbt = bbuf[1:].view(N, K)
            gbt.copy_(gpu(b.T.copy()))
            gb = gbt.t()                                  # B[k, n], k unit-stride
            ref = a.astype(np.float64) @ b.astype(np.float64)
            scale = np.abs(a).astype(np.float64) @ np.abs(b).astype(np.float64)
            for cfg in range(tn.tune_num_configs()):
                tn.tune_force_config(cfg)
                out = tn.contract_between(ga, gb, [1], [0], prec=prec)
                check(host(out), ref, scale, TOL[prec], f"{M}x{K}x{N} tile config {cfg}")
            # the same operands stored row-contiguous (M and N unit-stride,
            # odd extents, rows from a one-float offset): 16-byte loads of
            # four rows with an element-wise partial last block
            at = gpu(np.zeros(K * M + 1, dtype=np.float32))
            gat = at[1:].view(K, M)
            gat.copy_(gpu(a.T.copy()))
            bb = gpu(np.zeros(K * N + 1, dtype=np.float32))
            gbb = bb[1:].view(K, N)
            gbb.copy_(gpu(b))
            for cfg in range(tn.tune_num_configs()):
                tn.tune_force_config(cfg)
                out = tn.contract_between(gat.t(), gbb, [1], [0], prec=prec)
                check(host(out), ref, scale, TOL[prec], f"{M}x{K}x{N} row-contiguous, tile config {cfg}")
    finally:
        tn.tune_force_config(-1)


# the last six tile configurations are the lean-stage split-BF16 kernels
# (both operands through LDS; B private per wave; B private in two k
# groups), then the same three on the exchanged operands
LEAN_CFGS = [16, 17, 18, 19, 20, 21]


@pytest.mark.parametrize("layout", ["kn", "kk", "mk"])
@pytest.mark.parametrize("shape", [(197, 296, 259), (160, 32, 256), (5, 8, 7), (330, 1000, 520), (161, 64, 33)])
def test_lean_split_kernels(shape, layout):
    """Every lean-stage kernel, forced, on ragged tiles, a partial last k
    stage, A along k or along m, B along n or along k, a two-axis M group and
    a permuted output, against the oracle at the split-BF16 target.  Where a
    lean kernel does not take the problem (precision, layout) the general
    tile of the same shape runs."""
    assert tn.tune_num_configs() == 22
    M, K, N = shape
    rng = np.random.default_rng(M * 7 + K)
    m1 = 3 if M % 3 == 0 else 1
    a = f32(rng.standard_normal((M // m1, m1, K)))
    b = f32(rng.standard_normal((K, N)))
    if layout[0] == "k":   # M group of two axes in reverse memory order, k contiguous
        ga = gpu(a.transpose(1, 0, 2).copy()).permute(1, 0, 2)
    else:                  # m contiguous
        ga = gpu(a.transpose(2, 0, 1).copy()).permute(1, 2, 0)
    gb = gpu(b) if layout[1] == "n" else gpu(b.T.copy()).t()
    ref = oracle.tensordot(a, b, [2], [0])
    scale = abs_scale(a, b, [2], [0])
    try:
        for cfg in LEAN_CFGS:
            tn.tune_force_config(cfg)
            out = tn.contract_between(ga, gb, [2], [0], prec="split_bf16")
            check(host(out), ref, scale, TOL["split_bf16"], f"lean config {cfg}")
            outp = torch.empty((N, M // m1, m1), device=DEV)
            tn.contract_between(ga, gb, [2], [0], out=outp.permute(1, 2, 0), prec="split_bf16")
            check(host(outp.permute(1, 2, 0)), ref, scale, TOL["split_bf16"], f"lean config {cfg}, permuted output")
            out = tn.contract_between(ga, gb, [2], [0], prec="fp32")
            check(host(out), ref, scale, TOL["fp32"], f"lean config {cfg} in FP32 (general tile)")
    finally:
        tn.tune_force_config(-1)


@pytest.mark.parametrize("layout", ["kk", "mk", "km", "mm", "gen"])
@pytest.mark.parametrize("prec", ["fp32", "split_bf16"])
def test_operand_layouts(layout, prec):
    """A stored M-major or K-major, B stored N-major or K-major, and a gather case."""
    rng = np.random.default_rng(11)
    M, K, N = 260, 132, 196
    a = f32(rng.standard_normal((M, K)))
    b = f32(rng.standard_normal((K, N)))
    ga = gpu(a) if layout[0] == "k" else gpu(a.T.copy()).t()
    gb = gpu(b.T.copy()).t() if layout[-1] == "k" else gpu(b)
    if layout == "gen":
        big = gpu(np.zeros((M, 3 * K), dtype=np.float32))
        big[:, ::3] = gpu(a)
        ga = big[:, ::3]
    out = tn.contract_between(ga, gb, [1], [0], prec=prec)
    ref = a.astype(np.float64) @ b.astype(np.float64)
    check(host(out), ref, np.abs(a).astype(np.float64) @ np.abs(b), TOL[prec], layout)


@pytest.mark.parametrize("prec", ["fp32", "split_bf16", "bf16"])
def test_rank0_and_rank1_results(prec):
    rng = np.random.default_rng(13)
    v = f32(rng.standard_normal(100_003))
    w = f32(rng.standard_normal(100_003))
    d = tn.contract_between(gpu(v), gpu(w), [0], [0], prec=prec)
    ref = float(np.dot(v.astype(np.float64), w.astype(np.float64)))
    assert d.dim() == 0
    tol = TOL[prec] if prec != "bf16" else 2e-2
    assert abs(float(host(d)) - ref) <= tol * float(np.dot(np.abs(v), np.abs(w)))
    m = f32(rng.standard_normal((300, 517)))
    x = f32(rng.standard_normal(517))
    out = tn.contract_between(gpu(m), gpu(x), [1], [0], prec=prec)
    check(host(out), m.astype(np.float64) @ x, np.abs(m) @ np.abs(x), tol, "matvec")
    out = tn.contract_between(gpu(x), gpu(m.T.copy()), [0], [0], prec=prec)
    check(host(out), m.astype(np.float64) @ x, np.abs(m) @ np.abs(x), tol, "vecmat")
    t3 = f32(rng.standard_normal((5, 7, 6)))
    u3 = f32(rng.standard_normal((6, 5, 7)))
    out = tn.contract_between(gpu(t3), gpu(u3), [0, 1, 2], [1, 2, 0], prec=prec)
    ref = oracle.tensordot(t3, u3, [0, 1, 2], [1, 2, 0])
    assert abs(float(host(out)) - float(ref)) <= tol * float(oracle.tensordot(np.abs(t3), np.abs(u3), [0, 1, 2], [1, 2, 0]))


def test_scalar_operands_and_unit_dims():
    s = gpu(np.float32(3.0).reshape(()))
    v = gpu(np.arange(5, dtype=np.float32))
    out = tn.contract_between(s, v, [], [])
    np.testing.assert_array_equal(host(out), 3.0 * np.arange(5))
    a = f32(np.random.default_rng(3).standard_normal((1, 4, 1, 3)))
    b = f32(np.random.default_rng(4).standard_normal((3, 1, 2)))
    out = tn.contract_between(gpu(a), gpu(b), [3, 2], [0, 1])
    check(host(out), oracle.tensordot(a, b, [3, 2], [0, 1]), abs_scale(a, b, [3, 2], [0, 1]), 1e-5)


def test_deterministic_results():
    rng = np.random.default_rng(17)
    a, b = gpu(rng.standard_normal((333, 444))), gpu(rng.standard_normal((444, 222)))
    for prec in ("fp32", "split_bf16"):
        x = host(tn.contract_between(a, b, [1], [0], prec=prec))
        y = host(tn.contract_between(a, b, [1], [0], prec=prec))
        np.testing.assert_array_equal(x, y)


def test_tune_cache_file_round_trip(tmp_path):
    """A timed choice is appended to the cache file; a later process state
    that loads the file uses the stored tile without timing."""
    rng = np.random.default_rng(29)
    a, b = f32(rng.standard_normal((384, 256))), f32(rng.standard_normal((256, 320)))
    ref = a.astype(np.float64) @ b
    path = tmp_path / "tiles.txt"
    try:
        tn.tune(path, 1)
        out = tn.contract_between(gpu(a), gpu(b), [1], [0], prec="split_bf16")
        chosen = tn.tune_last_choice()
        lines = path.read_text().splitlines()
        assert len(lines) == 1 and lines[0].endswith(f"-> {chosen}"), lines
        check(host(out), ref, np.abs(a) @ np.abs(b), 1e-6, "timed")
        # point the stored entry at the 32 x 32 tile (id 7) and reload at level 0
        path.write_text(lines[0].rsplit("->", 1)[0] + "-> 7\n")
        tn.tune(path, 0)
        out = tn.contract_between(gpu(a), gpu(b), [1], [0], prec="split_bf16")
        assert tn.tune_last_choice() == 7
        check(host(out), ref, np.abs(a) @ np.abs(b), 1e-6, "from file")
    finally:
        tn.tune(None, 0)


def test_autotune_path_matches():
    rng = np.random.default_rng(19)
    a, b = f32(rng.standard_normal((384, 256))), f32(rng.standard_normal((256, 320)))
    ref = a.astype(np.float64) @ b
    try:
        tn.tune_set_level(1)
        out = tn.contract_between(gpu(a), gpu(b), [1], [0], prec="split_bf16")
        assert 0 <= tn.tune_last_choice() < tn.tune_num_configs()
        check(host(out), ref, np.abs(a) @ np.abs(b), 1e-6, "autotuned")
    finally:
        tn.tune_set_level(0)


# ---------------------------------------------------------------------------
# trace and outer products


@pytest.mark.parametrize("seed", range(6))
def test_trace_edge(seed):
    rng = np.random.default_rng(700 + seed)
    r = int(rng.integers(2, 6))
    shape = [int(rng.integers(1, 9)) for _ in range(r)]
    i, j = [int(x) for x in rng.permutation(r)[:2]]
    shape[j] = shape[i] = max(shape[i], 2) if seed % 2 else shape[i]
    a = f32(rng.standard_normal(shape))
    ga = permuted_input(a, rng)
    out = tn.trace_edge(ga, i, j)
    ref = oracle.trace_edge(a, i, j)
    check(host(out), ref, oracle.trace_edge(np.abs(a), i, j), 1e-6)


def test_trace_large_scalar():
    a = f32(np.random.default_rng(1).standard_normal((3001, 3001)))
    out = tn.trace_edge(gpu(a), 0, 1)
    ref = float(np.trace(a.astype(np.float64)))
    assert abs(float(host(out)) - ref) < 1e-6 * float(np.sum(np.abs(np.diag(a))))


def test_outer_product_strided():
    rng = np.random.default_rng(23)
    a = f32(rng.standard_normal((33, 7)))
    b = f32(rng.standard_normal((5, 65)))
    ga = gpu(a.T.copy()).t()
    out = tn.outer_product(ga, gpu(b))
    np.testing.assert_array_equal(host(out), oracle.outer_product(a, b).astype(np.float32))


# ---------------------------------------------------------------------------
# networks


def _small_network(rng):
    t0 = f32(rng.standard_normal((2, 3, 3, 2)))
    t1 = f32(rng.standard_normal((2, 2, 3)))
    t2 = f32(rng.standard_normal((2, 2, 2, 2)))
    t3 = f32(rng.standard_normal((2, 2)))
    return [t0, t1, t2, t3], [[0, 9, 9, 1], [0, 2, -2], [1, 2, 3, -1], [3, -3]]


def test_network_all_orders():
    rng = np.random.default_rng(31)
    ts, ls = _small_network(rng)
    ref = oracle.contract_network(ts, ls)
    gts = [gpu(t) for t in ts]
    for order in itertools.permutations([0, 1, 2, 3, 9]):
        out = tn.contract_network(gts, ls, order=list(order))
        np.testing.assert_allclose(host(out), ref, rtol=1e-5, atol=1e-5)


@pytest.mark.parametrize("prec", ["fp32", "split_bf16"])
def test_network_mps_ring(prec):
    # a periodic 6-site MPS contracted with itself: a closed network (scalar)
    rng = np.random.default_rng(37)
    n, chi = 6, 24
    sites = [f32(rng.standard_normal((chi, 2, chi)) / np.sqrt(2 * chi)) for _ in range(n)]
    ts = sites + sites
    labels = [[k, 100 + k, (k + 1) % n] for k in range(n)] + [[10 + k, 100 + k, 10 + (k + 1) % n] for k in range(n)]
    ref = oracle.contract_network(ts, labels)
    out = tn.contract_network([gpu(t) for t in ts], labels, prec=prec)
    assert abs(float(host(out)) / float(ref) - 1) < 10 * TOL[prec]


def test_network_single_node_permutation_and_disconnected():
    rng = np.random.default_rng(41)
    a = f32(rng.standard_normal((3, 4, 5)))
    out = tn.contract_network([gpu(a)], [[-2, -3, -1]])
    np.testing.assert_array_equal(host(out), np.transpose(a, (2, 0, 1)))
    b = f32(rng.standard_normal(6))
    out = tn.contract_network([gpu(a), gpu(b)], [[-2, -4, -1], [-3]])
    np.testing.assert_array_equal(host(out), oracle.contract_network([a, b], [[-2, -4, -1], [-3]]).astype(np.float32))
    c = f32(rng.standard_normal((4, 4)))
    out = tn.contract_network([gpu(c)], [[0, 0]])
    assert abs(float(host(out)) - float(np.trace(c))) < 1e-5


def _rounded_close(got, ref, absref, what):
    """FP64 sums rounded once to FP32: within half an FP32 ulp of the exact
    value plus the FP64 summation error (K * 2^-53 of the absolute sum)."""
    got = np.asarray(got, dtype=np.float64)
    err = np.abs(got - ref)
    bound = 2.0 ** -24 * np.abs(ref) + 1e-9 * absref + 1e-30
    assert np.all(err <= bound), (what, float(np.max(err / bound)))


def _contract_raw(a, b, axes_a, axes_b, out, ws):
    """The C entry point with an explicit workspace (None: no scratch)."""
    import ctypes as C
    from paper_1905_01330_amd import _lib as Lb

    da, db, do = Lb.tensor_desc(a), Lb.tensor_desc(b), Lb.tensor_desc(out)
    Lb.check(Lb.lib().tn_contract_between(C.byref(da), C.byref(db), len(axes_a), Lb.int_array(axes_a),
                                          Lb.int_array(axes_b), C.byref(do),
                                          C.c_void_p(ws.data_ptr()) if ws is not None else None,
                                          ws.numel() if ws is not None else 0, 0, Lb.stream_ptr()))
    return out


@pytest.mark.parametrize("with_scratch", [True, False])
def test_long_sums_split_and_fallback(with_scratch):
    """Dot products and few-row matrix-vector products with long, ragged,
    misaligned sums: split over workgroups (scratch) or one workgroup per
    sum (no scratch); both give the FP64 sum rounded once, bit-identically
    on repeated calls."""
    rng = np.random.default_rng(21)
    ws = torch.empty(tn._lib.REDUCE_WORKSPACE_BYTES, dtype=torch.uint8, device=DEV) if with_scratch else None
    n = (1 << 22) + 3
    v = f32(rng.standard_normal(n + 1))
    w = f32(rng.standard_normal(n + 1))
    gv, gw = gpu(v), gpu(w)
    for off in (0, 1):   # off = 1: rows not 16-byte aligned
        x, y = gv[off:off + n], gw[off:off + n]
        out = torch.empty((), device=DEV)
        _contract_raw(x, y, [0], [0], out, ws)
        first = host(out).copy()
        _contract_raw(x, y, [0], [0], out, ws)
        assert np.array_equal(first, host(out)), "repeated call differs"
        xs, ys = v[off:off + n].astype(np.float64), w[off:off + n].astype(np.float64)
        _rounded_close(first, float(np.dot(xs, ys)), float(np.dot(np.abs(xs), np.abs(ys))), f"dot off={off}")
    m = f32(rng.standard_normal((7, 200_003)))
    x = f32(rng.standard_normal(200_003))
    out = torch.empty(7, device=DEV)
    _contract_raw(gpu(m), gpu(x), [1], [0], out, ws)
    m64, x64 = m.astype(np.float64), x.astype(np.float64)
    _rounded_close(host(out), m64 @ x64, np.abs(m64) @ np.abs(x64), "few-row matvec")


def test_reduction_layout_paths():
    """Many long rows (wavefront per row, 16-byte loads, ragged tail), column
    sums (thread per output), traces over leading and outer axes, outer
    products with four outputs per thread, odd extents and misaligned or
    permuted outputs: all exact to one FP32 rounding of the FP64 sum."""
    rng = np.random.default_rng(22)
    m = f32(rng.standard_normal((3000, 1031)))
    x = f32(rng.standard_normal(1031))
    m64, x64 = m.astype(np.float64), x.astype(np.float64)
    out = tn.contract_between(gpu(m), gpu(x), [1], [0])
    _rounded_close(host(out), m64 @ x64, np.abs(m64) @ np.abs(x64), "matvec rows")
    y = f32(rng.standard_normal(3000))
    out = tn.contract_between(gpu(y), gpu(m), [0], [0])
    y64 = y.astype(np.float64)
    _rounded_close(host(out), y64 @ m64, np.abs(y64) @ np.abs(m64), "column sums")
    t = f32(rng.standard_normal((8, 8, 1003)))
    out = tn.trace_edge(gpu(t), 0, 1)
    _rounded_close(host(out), oracle.trace_edge(t.astype(np.float64), 0, 1),
                   oracle.trace_edge(np.abs(t).astype(np.float64), 0, 1), "trace leading axes")
    t = f32(rng.standard_normal((8, 8, 1024)))
    for view in (slice(0, 1024), slice(1, 1001)):      # four outputs per thread: aligned, misaligned
        out = tn.trace_edge(gpu(t)[:, :, view], 0, 1)
        tv = t[:, :, view].astype(np.float64)
        _rounded_close(host(out), oracle.trace_edge(tv, 0, 1), oracle.trace_edge(np.abs(tv), 0, 1), "trace x4")
    t = f32(rng.standard_normal((6, 1001, 6)))
    out = tn.trace_edge(gpu(t), 0, 2)
    _rounded_close(host(out), oracle.trace_edge(t.astype(np.float64), 0, 2),
                   oracle.trace_edge(np.abs(t).astype(np.float64), 0, 2), "trace outer axes")
    # few output quads: four threads share each quad, each over every fourth k
    # (32 diagonal terms; 20 terms, not a multiple of four; a ragged last workgroup)
    for shape in ((32, 32, 4096), (20, 20, 2048), (16, 16, 1028)):
        t = f32(rng.standard_normal(shape))
        out = tn.trace_edge(gpu(t), 0, 1)
        _rounded_close(host(out), oracle.trace_edge(t.astype(np.float64), 0, 1),
                       oracle.trace_edge(np.abs(t).astype(np.float64), 0, 1), f"trace k-split {shape}")
    for na, nb in ((37, 1024), (5, 1023), (3, 4)):
        a = f32(rng.standard_normal(na))
        b = f32(rng.standard_normal(nb))
        ref = oracle.outer_product(a.astype(np.float64), b.astype(np.float64))
        out = tn.outer_product(gpu(a), gpu(b))
        np.testing.assert_array_equal(host(out), ref.astype(np.float32))
        buf = torch.empty(na * nb + 1, device=DEV)
        mis = buf[1:].view(na, nb)             # 4-byte aligned only
        tn.outer_product(gpu(a), gpu(b), out=mis)
        np.testing.assert_array_equal(host(mis), ref.astype(np.float32))
        tr = torch.empty((nb, na), device=DEV)
        tn.outer_product(gpu(a), gpu(b), out=tr.t())   # permuted store
        np.testing.assert_array_equal(host(tr).T, ref.astype(np.float32))


def test_network_ending_in_a_long_dot():
    """A network whose last step is a long dot product takes the split sum
    from the network workspace."""
    rng = np.random.default_rng(23)
    a = f32(rng.standard_normal((256, 300)))
    b = f32(rng.standard_normal((300, 256)))
    c = f32(rng.standard_normal((256, 256)))
    out = tn.contract_network([gpu(a), gpu(b), gpu(c)], [[0, 1], [1, 2], [2, 0]], order=[1, 2, 0])
    ab = a.astype(np.float64) @ b.astype(np.float64)
    ref = float(np.sum(ab * c.astype(np.float64).T))
    scale = float(np.sum((np.abs(a).astype(np.float64) @ np.abs(b)) * np.abs(c).T))
    assert abs(float(host(out)) - ref) <= 1e-5 * scale


@pytest.mark.parametrize("prec", ["fp32", "split_bf16", "bf16"])
def test_tiny_contracted_and_free_extents(prec):
    """An MPO acting on a bond pair (K = 10, N = 10 over a large M), its
    transpose (M = 10), K = 32 / N = 16 at the limit, strided views and a
    permuted output: the HBM-bound small path, against the oracle."""
    rng = np.random.default_rng(24)
    tol = TOL[prec]
    t1 = f32(rng.standard_normal((64, 5, 2, 96)))        # [a', u, s, b]
    w = f32(rng.standard_normal((5, 5, 2, 2)))           # [u, v, t, s]
    out = tn.contract_between(gpu(t1), gpu(w), [1, 2], [0, 3], prec=prec)
    check(host(out), oracle.tensordot(t1, w, [1, 2], [0, 3]), abs_scale(t1, w, [1, 2], [0, 3]), tol, "mpo step")
    out = tn.contract_between(gpu(w), gpu(t1), [0, 3], [1, 2], prec=prec)
    check(host(out), oracle.tensordot(w, t1, [0, 3], [1, 2]), abs_scale(w, t1, [0, 3], [1, 2]), tol, "transposed")
    a = f32(rng.standard_normal((3000, 32)))
    b = f32(rng.standard_normal((32, 16)))
    big = gpu(np.zeros((3000, 64), dtype=np.float32))
    big[:, ::2] = gpu(a)
    res = torch.empty((16, 3000), device=DEV)
    tn.contract_between(big[:, ::2], gpu(b), [1], [0], out=res.t(), prec=prec)
    check(host(res).T, a.astype(np.float64) @ b, np.abs(a).astype(np.float64) @ np.abs(b), tol, "strided, permuted out")


@pytest.mark.parametrize("method", ["greedy", "optimal"])
def test_network_with_searched_order(method):
    """A six-node network with a trace, a double edge and open legs,
    contracted in the searched order: equal to the oracle's (any order gives
    the same tensor up to rounding)."""
    rng = np.random.default_rng(25)
    labels = [[0, 1, 7, 7], [1, 2, -1], [2, 3, 4], [3, 4, 5, -2], [5, 6], [6, 0, -3]]
    dims = {0: 6, 1: 7, 2: 5, 3: 4, 4: 3, 5: 8, 6: 9, 7: 2, -1: 3, -2: 5, -3: 4}
    ts = [f32(rng.standard_normal([dims[l] for l in ls]) / 3) for ls in labels]
    ref = oracle.contract_network([t.astype(np.float64) for t in ts], labels)
    order, flops = tn.network_order([gpu(t) for t in ts], labels, method)
    assert flops > 0 and order[0] == 7
    out = tn.contract_network([gpu(t) for t in ts], labels, order=method)
    scale = oracle.contract_network([np.abs(t).astype(np.float64) for t in ts], labels)
    check(host(out), ref, scale, 1e-5, f"network {method}")


@pytest.mark.parametrize("prec", ["fp32", "split_bf16", "bf16"])
def test_row_contiguous_operands_of_odd_extent(prec):
    """Operands whose free index is unit-stride but of odd extent or not
    16-byte aligned: the row-contiguous gathers with scalar loads."""
    rng = np.random.default_rng(26)
    M, K, N = 261, 133, 197
    a = f32(rng.standard_normal((M, K)))
    b = f32(rng.standard_normal((K, N)))
    ga = gpu(a.T.copy()).t()                       # M unit-stride, M odd
    buf = gpu(np.zeros(K * N + 1, dtype=np.float32))
    gb = buf[1:].view(K, N)                        # N unit-stride, misaligned rows
    gb.copy_(gpu(b))
    ref = a.astype(np.float64) @ b.astype(np.float64)
    scale = np.abs(a).astype(np.float64) @ np.abs(b).astype(np.float64)
    out = tn.contract_between(ga, gb, [1], [0], prec=prec)
    check(host(out), ref, scale, TOL[prec], "odd row-contiguous")
