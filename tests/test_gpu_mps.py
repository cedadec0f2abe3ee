"""GPU parity of the chain-network entry points (MPS inner products, the
uneven batch, the environment sweep and the FP64 canonicalisation) against
the FP64 oracle, plus full-size checks through properties that hold exactly.

Inner products of independent random chains cancel strongly, so those are
gated on the Cauchy-Schwarz scale |x - x_ref| / (|psi| |phi|); correlated
pairs (phi = psi + 0.1 G) are gated relatively.
"""
import math

import numpy as np
import pytest
import torch

import oracle
import paper_1905_01330_amd as tn
from helpers import energy_abs_scale, product_state_mps, spin_angle_vector
from paper_1905_01330_amd import inputs

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")
TOL = {"fp32": 1e-5, "split_bf16": 1e-6}


def g32(xs):
    return [torch.tensor(np.asarray(x, dtype=np.float32), device=DEV) for x in xs]


def r32(xs):
    return [np.asarray(x, dtype=np.float32).astype(np.float64) for x in xs]


def ms(t):
    torch.cuda.synchronize()
    v = t.cpu().numpy()
    return float(v[0]), float(v[1])


def value_rel(m, s, mr, sr):
    return abs(m / mr * math.exp(s - sr) - 1.0)


@pytest.mark.parametrize("prec", ["fp32", "split_bf16"])
def test_inner_cfg1(prec):
    psi = r32(inputs.random_mps(16, 2, 16, 101))
    phi = r32(inputs.random_mps(16, 2, 16, 102))
    mr, sr = oracle.mps_inner(psi, phi)
    m, s = ms(tn.mps_inner(g32(psi), g32(phi), prec=prec))
    npsi = math.sqrt(oracle.mps_inner_value(psi, psi))
    nphi = math.sqrt(oracle.mps_inner_value(phi, phi))
    assert abs(m * math.exp(s) - mr * math.exp(sr)) / (npsi * nphi) <= TOL[prec]
    for x in (psi, phi):
        mr2, sr2 = oracle.mps_inner(x, x)
        m2, s2 = ms(tn.mps_inner(g32(x), g32(x), prec=prec))
        assert value_rel(m2, s2, mr2, sr2) <= TOL[prec]


@pytest.mark.parametrize("prec", ["fp32", "split_bf16"])
def test_inner_correlated_pair(prec):
    psi, phi = inputs.correlated_mps_pair(60, 2, 96, 403)
    psi, phi = r32(psi), r32(phi)
    mr, sr = oracle.mps_inner(psi, phi)
    m, s = ms(tn.mps_inner(g32(psi), g32(phi), prec=prec))
    assert value_rel(m, s, mr, sr) <= TOL[prec]


@pytest.mark.parametrize("prec", ["fp32", "split_bf16"])
def test_inner_k_slices(prec, tmp_path):
    """The two-ended inner product's GEMMs cut into 2 and into 4 k-slices
    (tile-cache entries rewritten with the slice count, loaded at level 0):
    the ket-site GEMM's 2^-e scale and the bra-site GEMM's |C| maximum move
    to the kernel that adds the slices.  On a chain whose raw value is far
    beyond FP32 (so every step's rescaling matters) the values match the
    oracle, and two slices change the result's low bits (the path ran)."""
    psi, phi = inputs.correlated_mps_pair(40, 2, 128, 409)
    psi, phi = [x * 32.0 for x in r32(psi)], r32(phi)
    mr, sr = oracle.mps_inner(psi, phi)
    assert sr > 88.0
    gp, gq = g32(psi), g32(phi)
    path = tmp_path / "tiles.txt"
    got = {}
    try:
        tn.tune(path, 1)
        ms(tn.mps_inner(gp, gq, prec=prec))   # fills the cache
        lines = [x for x in path.read_text().splitlines() if x and not x.startswith("G ")]
        assert lines
        for lg in (0, 1, 2):
            forced = tmp_path / f"tiles{lg}.txt"
            forced.write_text("".join(
                f"{x.split('->')[0].strip()} -> {int(x.split('->')[1]) % 100 + 100 * lg}\n" for x in lines))
            tn.tune(forced, 0)
            got[lg] = ms(tn.mps_inner(gp, gq, prec=prec))
    finally:
        tn.tune(None, 0)
    for lg, (m, s) in got.items():
        assert value_rel(m, s, mr, sr) <= TOL[prec], (lg, m, s, mr, sr)
    assert got[1] != got[0]


def test_inner_rescaling_over_long_chain():
    # entries 4x larger than normalised: the raw value would overflow FP32 by far
    psi = [x * 4.0 for x in r32(inputs.random_mps(200, 2, 32, 9))]
    mr, sr = oracle.mps_inner(psi, psi)
    assert sr > 100.0
    m, s = ms(tn.mps_inner(g32(psi), g32(psi)))
    assert value_rel(m, s, mr, sr) <= 2e-5


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 7])
def test_inner_short_and_odd_chains(n):
    """Below four sites the chain runs from the left only; from four on the
    halves run from both ends and meet at bond n // 2 (odd n: unequal halves)."""
    psi = r32(inputs.random_mps(n, 2, 8, 500 + n))
    phi = r32(inputs.random_mps(n, 2, 8, 600 + n))
    mr, sr = oracle.mps_inner(psi, phi)
    m, s = ms(tn.mps_inner(g32(psi), g32(phi)))
    npsi = math.sqrt(oracle.mps_inner_value(psi, psi))
    nphi = math.sqrt(oracle.mps_inner_value(phi, phi))
    assert abs(m * math.exp(s) - mr * math.exp(sr)) / (npsi * nphi) <= TOL["fp32"]


def test_inner_exactly_zero():
    """Orthogonal product states (bond dimension 1): the middle-bond sum is an
    exact zero, which the mantissa/scale form must carry as m = 0."""
    n = 6
    zero = [np.array([1.0, 0.0]).reshape(1, 2, 1) for _ in range(n)]
    one = [x.copy() for x in zero]
    one[3] = np.array([0.0, 1.0]).reshape(1, 2, 1)
    for prec in ("fp32", "split_bf16"):
        m, s = ms(tn.mps_inner(g32(zero), g32(one), prec=prec))
        assert m == 0.0 and np.isfinite(s)
        m, s = ms(tn.mps_inner(g32(zero), g32(zero), prec=prec))
        assert abs(m * math.exp(s) - 1.0) < 1e-12
    out = tn.mps_inner_batched([(g32(zero), g32(one)), (g32(zero), g32(zero))]).cpu().numpy()
    assert out[0, 0] == 0.0 and abs(out[1, 0] * math.exp(out[1, 1]) - 1.0) < 1e-12


def test_inner_product_state_norm_one():
    rng = np.random.default_rng(3)
    n = 40
    vecs = []
    for _ in range(n):
        v = rng.standard_normal(2)
        vecs.append(v / np.linalg.norm(v))
    sites = product_state_mps(vecs, inputs.bond_dims(n, 2, 64), rng)
    m, s = ms(tn.mps_inner(g32(sites), g32(sites), prec="split_bf16"))
    assert abs(m * math.exp(s) - 1.0) < 2e-6


@pytest.mark.parametrize("prec", ["fp32", "split_bf16"])
def test_inner_batched_uneven(prec):
    shapes = inputs.uneven_chain_shapes(24, 403, n_range=(4, 40), chi_range=(2, 70))
    chains, refs = [], []
    for i, (n, chi) in enumerate(shapes):
        psi, phi = inputs.uneven_chain(i, n, chi)
        psi, phi = r32(psi), r32(phi)
        refs.append(oracle.mps_inner(psi, phi))
        chains.append((g32(psi), g32(phi)))
    out = tn.mps_inner_batched(chains, prec=prec)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    for i, (mr, sr) in enumerate(refs):
        assert value_rel(got[i, 0], got[i, 1], mr, sr) <= 4 * TOL[prec], (i, shapes[i])
    # single-chain path agrees with the batch
    m, s = ms(tn.mps_inner(chains[5][0], chains[5][1], prec=prec))
    assert value_rel(m, s, got[5, 0], got[5, 1]) <= 4 * TOL[prec]


@pytest.mark.parametrize("prec", ["fp32", "split_bf16"])
def test_inner_batched_aligned_bonds(prec):
    """Bond dimensions that are multiples of four: the grouped launches take
    the fast gathers."""
    rng = np.random.default_rng(31)
    chains, refs = [], []
    for i in range(12):
        n, chi = int(rng.integers(6, 30)), int(rng.choice([8, 16, 32, 64, 128]))
        psi, phi = inputs.uneven_chain(i, n, chi, seed=409)
        psi, phi = r32(psi), r32(phi)
        refs.append(oracle.mps_inner(psi, phi))
        chains.append((g32(psi), g32(phi)))
    out = tn.mps_inner_batched(chains, prec=prec)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    for i, (mr, sr) in enumerate(refs):
        assert value_rel(got[i, 0], got[i, 1], mr, sr) <= 4 * TOL[prec], i


@pytest.mark.parametrize("prec", ["fp32", "split_bf16"])
@pytest.mark.parametrize("tile", [0, 1, 2, 3, 4])
def test_inner_batched_every_grouped_tile(tile, prec):
    """Each grouped tile (128, 64, 32, 64 in two k-slices, 160 x 256) on odd and aligned
    bonds, with several tiles per problem and ragged edges."""
    rng = np.random.default_rng(53)
    chains, refs = [], []
    for i, chi in enumerate([3, 17, 64, 97, 150, 200]):
        n = int(rng.integers(5, 12))
        psi, phi = inputs.uneven_chain(i, n, chi, seed=421)
        psi, phi = r32(psi), r32(phi)
        refs.append(oracle.mps_inner(psi, phi))
        chains.append((g32(psi), g32(phi)))
    try:
        tn.tune_force_grouped_config(tile)
        out = tn.mps_inner_batched(chains, prec=prec)
        torch.cuda.synchronize()
    finally:
        tn.tune_force_grouped_config(-1)
    got = out.cpu().numpy()
    for i, (mr, sr) in enumerate(refs):
        assert value_rel(got[i, 0], got[i, 1], mr, sr) <= 4 * TOL[prec], (tile, i)


@pytest.mark.parametrize("prec", ["fp32", "split_bf16"])
def test_inner_batched_tuned_steps(prec, tmp_path):
    """With tuning on, the first launch times the grouped tiles on every
    step (re-running a step's launch on its real inputs) and records one
    choice per step signature and precision in the cache file; the results
    match the oracle.  Later launches are served from the cache: the one
    after a reload of the file times and appends nothing and repeats the
    previous cached launch exactly."""
    rng = np.random.default_rng(59)
    chains, refs = [], []
    for i, chi in enumerate([5, 24, 64, 130]):
        n = int(rng.integers(6, 14))
        psi, phi = inputs.uneven_chain(i, n, chi, seed=431)
        psi, phi = r32(psi), r32(phi)
        refs.append(oracle.mps_inner(psi, phi))
        chains.append((g32(psi), g32(phi)))
    path = tmp_path / "tiles.txt"
    try:
        tn.tune(path, 1)
        out = tn.mps_inner_batched(chains, prec=prec)
        torch.cuda.synchronize()
        lines = [x for x in path.read_text().splitlines() if x.startswith("G ")]
        assert lines, "no grouped choices recorded"
        assert all(int(x.rsplit("->", 1)[1]) in (0, 1, 2, 3, 4) for x in lines)
        assert all(int(x.split()[2]) == {"fp32": 0, "split_bf16": 2}[prec] for x in lines)
        again = tn.mps_inner_batched(chains, prec=prec)
        torch.cuda.synchronize()
        n_lines = len(lines)
        tn.tune(path, 1)   # reload: every step is cached, nothing is timed or appended
        third = tn.mps_inner_batched(chains, prec=prec)
        torch.cuda.synchronize()
        assert len([x for x in path.read_text().splitlines() if x.startswith("G ")]) == n_lines
        np.testing.assert_array_equal(again.cpu().numpy(), third.cpu().numpy())
    finally:
        tn.tune(None, 0)
    for res in (out, again):
        got = res.cpu().numpy()
        for i, (mr, sr) in enumerate(refs):
            assert value_rel(got[i, 0], got[i, 1], mr, sr) <= 4 * TOL[prec], i


# ---------------------------------------------------------------------------
# environment sweeps


def canonical(n, chi, seed):
    can, _ = oracle.left_canonicalize(inputs.random_mps(n, 2, chi, seed))
    return r32(can)


def env_errors(ls, rs, ls_ref, rs_ref):
    """Max relative Frobenius error over the environment tensors L_1..L_{N-1}
    and R_1..R_{N-1} (L_N and R_0 are the energy, checked on its own scale)."""
    n = len(ls) - 1
    el = max(np.linalg.norm(ls[k].cpu().double().numpy() - ls_ref[k]) / np.linalg.norm(ls_ref[k]) for k in range(1, n))
    er = max(np.linalg.norm(rs[k].cpu().double().numpy() - rs_ref[k]) / np.linalg.norm(rs_ref[k]) for k in range(1, n))
    return el, er


@pytest.mark.parametrize("model", ["tfim", "xxz"])
@pytest.mark.parametrize("prec", ["fp32", "split_bf16"])
def test_env_sweep_vs_oracle(model, prec):
    n, chi = 24, 64
    psi = canonical(n, chi, 201)
    mpo = inputs.tfim_mpo(n) if model == "tfim" else inputs.xxz_mpo(n, 0.5)
    ls_ref, rs_ref, el, er = oracle.env_sweep(psi, mpo)
    ls, rs, e = tn.mps_env_sweep(g32(psi), g32(mpo), prec=prec)
    torch.cuda.synchronize()
    errl, errr = env_errors(ls, rs, ls_ref, rs_ref)
    tol = TOL[prec]
    assert errl <= tol and errr <= tol, (errl, errr, tol)
    e = e.cpu().numpy()
    sl, sr = energy_abs_scale(psi, mpo, ls_ref, rs_ref)
    assert abs(e[0] - el) <= tol * sl and abs(e[1] - er) <= tol * sr, (e, el, er, sl, sr)
    if prec == "split_bf16":
        # the compensated products must not be less accurate than the FP32 path
        ls32, rs32, _ = tn.mps_env_sweep(g32(psi), g32(mpo), prec="fp32")
        torch.cuda.synchronize()
        e32l, e32r = env_errors(ls32, rs32, ls_ref, rs_ref)
        assert errl <= 1.2 * e32l and errr <= 1.2 * e32r, (errl, errr, e32l, e32r)


def test_concurrent_calls_on_several_streams():
    """Two-direction sweeps and two-ended inner products issued on three
    caller streams at once (each forks to the side stream assigned to its
    stream) give the same results, bit for bit, as the same calls made one
    after another on the default stream."""
    n, chi = 24, 64
    psi = canonical(n, chi, 211)
    mpo = inputs.xxz_mpo(n, 0.5)
    gp, gm = g32(psi), g32(mpo)
    ref_sweep = tn.mps_env_sweep(gp, gm, prec="split_bf16")
    ref_inner = tn.mps_inner(gp, gp, prec="fp32")
    torch.cuda.synchronize()
    streams = [torch.cuda.Stream() for _ in range(3)]
    outs = []
    for rep in range(2):
        for st in streams:
            st.wait_stream(torch.cuda.current_stream())
            with torch.cuda.stream(st):
                outs.append((tn.mps_env_sweep(gp, gm, prec="split_bf16"), tn.mps_inner(gp, gp, prec="fp32")))
    torch.cuda.synchronize()
    for (ls, rs, e), inner in outs:
        for k in range(n + 1):
            assert torch.equal(ls[k], ref_sweep[0][k]) and torch.equal(rs[k], ref_sweep[1][k]), k
        assert torch.equal(e, ref_sweep[2])
        assert torch.equal(inner, ref_inner)


@pytest.mark.parametrize("prec", ["fp32", "split_bf16"])
def test_env_sweep_tuned_shared_chip(prec, tmp_path):
    """With tuning on, the GEMMs of a two-direction sweep, which share the
    chip with the other direction, are timed as pairs and recorded under a
    key of their own (1000 added to the groups field); the same GEMMs in a
    one-direction sweep are recorded apart.  Results match the oracle, and
    after a reload of the file every choice is served from it (nothing is
    appended) with bit-identical results."""
    n, chi = 16, 96
    psi = canonical(n, chi, 223)
    mpo = inputs.xxz_mpo(n, 0.5)
    ls_ref, rs_ref, _, _ = oracle.env_sweep(psi, mpo)
    gp, gm = g32(psi), g32(mpo)
    path = tmp_path / "tiles.txt"

    def keys():
        return [x.split("->")[0].split() for x in path.read_text().splitlines() if x and not x.startswith("G ")]

    try:
        tn.tune(path, 1)
        ls, rs, e = tn.mps_env_sweep(gp, gm, prec=prec)
        torch.cuda.synchronize()
        both = keys()
        assert both and all(int(k[8]) >= 1000 for k in both), both
        ls1, _, _ = tn.mps_env_sweep(gp, gm, right=False, prec=prec)
        torch.cuda.synchronize()
        one = keys()[len(both):]
        assert one and all(int(k[8]) < 1000 for k in one), one
        n_lines = len(keys())
        tn.tune(path, 1)   # reload
        ls2, rs2, e2 = tn.mps_env_sweep(gp, gm, prec=prec)
        torch.cuda.synchronize()
        assert len(keys()) == n_lines
    finally:
        tn.tune(None, 0)
    errl, errr = env_errors(ls, rs, ls_ref, rs_ref)
    assert errl <= TOL[prec] and errr <= TOL[prec], (errl, errr)
    errl1, _ = env_errors(ls1, rs, ls_ref, rs_ref)
    assert errl1 <= TOL[prec], errl1
    for k in range(n + 1):
        assert torch.equal(ls[k], ls2[k]) and torch.equal(rs[k], rs2[k]), k
    assert torch.equal(e, e2)


@pytest.mark.parametrize("prec", ["fp32", "split_bf16"])
def test_env_sweep_k_slices(prec, tmp_path):
    """The sweep's GEMMs cut into 2 and into 4 k-slices (tile-cache entries
    rewritten with the slice count: choice = tile + 100 log2(slices), loaded
    at level 0 so nothing is re-timed) give environments within the oracle
    tolerance; with two slices, which every bulk GEMM of this chain can
    take, the sums run in another order than the whole GEMMs' (the results
    differ from theirs in low bits).  Slice counts a GEMM cannot take (K too
    short) fall back to the whole GEMM."""
    n, chi = 16, 128   # bonds 1, 2, 4, ..., 128, 128, 128, ..., 2, 1
    psi = canonical(n, chi, 227)
    mpo = inputs.xxz_mpo(n, 0.5)
    ls_ref, rs_ref, el, er = oracle.env_sweep(psi, mpo)
    gp, gm = g32(psi), g32(mpo)
    path = tmp_path / "tiles.txt"
    outs = {}
    try:
        tn.tune(path, 1)
        tn.mps_env_sweep(gp, gm, prec=prec)   # fills the cache
        torch.cuda.synchronize()
        lines = [x for x in path.read_text().splitlines() if x and not x.startswith("G ")]
        assert lines
        for lg in (0, 1, 2):
            forced = tmp_path / f"tiles{lg}.txt"
            forced.write_text("".join(
                f"{x.split('->')[0].strip()} -> {int(x.split('->')[1]) % 100 + 100 * lg}\n" for x in lines))
            tn.tune(forced, 0)
            outs[lg] = tn.mps_env_sweep(gp, gm, prec=prec)
            torch.cuda.synchronize()
    finally:
        tn.tune(None, 0)
    for lg, (ls, rs, e) in outs.items():
        errl, errr = env_errors(ls, rs, ls_ref, rs_ref)
        assert errl <= TOL[prec] and errr <= TOL[prec], (lg, errl, errr)
        sl, sr = energy_abs_scale(psi, mpo, ls_ref, rs_ref)
        e = e.cpu().numpy()
        assert abs(e[0] - el) <= TOL[prec] * sl and abs(e[1] - er) <= TOL[prec] * sr, (lg, e, el, er)
    assert any(not torch.equal(outs[1][0][k], outs[0][0][k]) for k in range(1, n))


def test_env_sweep_cfg2_full():
    """N = 100, chi = 256, TFIM (J = g = 1), canonical random MPS: FP32 vs the oracle."""
    n, chi = 100, 256
    psi = canonical(n, chi, 201)
    mpo = inputs.tfim_mpo(n)
    ls_ref, rs_ref, el, er = oracle.env_sweep(psi, mpo)
    ls, rs, e = tn.mps_env_sweep(g32(psi), g32(mpo), prec="fp32")
    torch.cuda.synchronize()
    errl, errr = env_errors(ls, rs, ls_ref, rs_ref)
    assert errl <= 1e-5 and errr <= 1e-5, (errl, errr)
    e = e.cpu().numpy()
    sl, sr = energy_abs_scale(psi, mpo, ls_ref, rs_ref)
    assert abs(e[0] - el) <= 1e-5 * sl and abs(e[1] - er) <= 1e-5 * sr, (e, el, er)


@pytest.mark.parametrize("prec", ["fp32", "split_bf16"])
def test_env_sweep_product_state_closed_forms(prec):
    rng = np.random.default_rng(55)
    n, chi = 30, 128
    dims = inputs.bond_dims(n, 2, chi)
    th = rng.uniform(0, 2 * np.pi, n)
    sites = product_state_mps([spin_angle_vector(t) for t in th], dims, rng)
    J, g = 1.0, 0.8
    ref = -J * sum(math.cos(th[i]) * math.cos(th[i + 1]) for i in range(n - 1)) - g * sum(math.sin(t) for t in th)
    _, _, e = tn.mps_env_sweep(g32(sites), g32(inputs.tfim_mpo(n, J, g)), store=False, prec=prec)
    e = e.cpu().numpy()
    assert abs(e[0] - ref) <= 2 * TOL[prec] * n and abs(e[1] - ref) <= 2 * TOL[prec] * n


def test_env_sweep_single_direction_and_strided_outputs():
    n, chi = 12, 16
    psi = canonical(n, chi, 5)
    mpo = inputs.xxz_mpo(n, 0.5)
    ls_ref, _, el, _ = oracle.env_sweep(psi, mpo)
    sweep = tn.EnvSweep(g32(psi), g32(mpo), left=True, right=False, store=True)
    # replace the stored outputs by permuted views
    bufs = [torch.empty((x.shape[2], x.shape[1], x.shape[0]), device=DEV) for x in sweep.L]
    sweep.L = [b.permute(2, 1, 0) for b in bufs]
    from paper_1905_01330_amd import _lib
    sweep.dL = _lib.tensor_array(sweep.L)
    sweep.run()
    torch.cuda.synchronize()
    for a, b in zip(sweep.L, ls_ref):
        np.testing.assert_allclose(a.cpu().double().numpy(), b, rtol=1e-4, atol=1e-5)
    assert abs(sweep.energy.cpu().numpy()[0] - el) < 1e-5 * max(1, abs(el))


# ---------------------------------------------------------------------------
# canonicalisation (FP64 on the GPU)


def test_left_canonicalize_matches_oracle():
    raw = inputs.random_mps(20, 2, 64, 201)
    ref, lognorm_ref = oracle.left_canonicalize(raw)
    sites = [torch.tensor(x, dtype=torch.float64, device=DEV) for x in raw]
    ln = tn.mps_left_canonicalize(sites)
    torch.cuda.synchronize()
    assert abs(float(ln.cpu()) - lognorm_ref) < 1e-12 * max(1, abs(lognorm_ref))
    for a, b in zip(sites, ref):
        np.testing.assert_allclose(a.cpu().numpy(), b, atol=1e-11)
        dk, d, dn = b.shape
        q = a.cpu().numpy().reshape(dk * d, dn)
        np.testing.assert_allclose(q.T @ q, np.eye(dn), atol=1e-12)


def test_left_canonicalize_blocked_and_column_paths():
    """Bonds that are not multiples of the 16-column panel, and two sites of
    more than 2048 rows (the column-by-column path), against the oracle."""
    dims = [1, 2, 4, 8, 13, 26, 50, 99, 190, 380, 700, 1100, 1200, 600, 300, 150, 75, 37, 18, 9, 4, 2, 1]
    raw = inputs.random_mps(len(dims) - 1, 2, 1024, 207, dims=dims)
    ref, lognorm_ref = oracle.left_canonicalize(raw)
    sites = [torch.tensor(x, dtype=torch.float64, device=DEV) for x in raw]
    ln = tn.mps_left_canonicalize(sites)
    torch.cuda.synchronize()
    assert abs(float(ln.cpu()) - lognorm_ref) < 1e-10 * max(1, abs(lognorm_ref))
    for k, (a, b) in enumerate(zip(sites, ref)):
        got = a.cpu().numpy()
        np.testing.assert_allclose(got, b, atol=1e-9, err_msg=f"site {k}")
        dk, d, dn = b.shape
        q = got.reshape(dk * d, dn)
        np.testing.assert_allclose(q.T @ q, np.eye(dn), atol=1e-11, err_msg=f"site {k}")


# ---------------------------------------------------------------------------
# full-size operator sweep (chi = 1024, N = 64, XXZ bond 5) through exact properties


@pytest.mark.parametrize("prec", ["fp32", "split_bf16"])
def test_env_sweep_chi1024_product_state(prec):
    """Neel state hidden by random orthogonal gauges at chi = 1024: E = -delta (N-1)/4."""
    rng = np.random.default_rng(301)
    n, chi, delta = 64, 1024, 0.5
    dims = inputs.bond_dims(n, 2, chi)
    up, dn = np.array([1.0, 0.0]), np.array([0.0, 1.0])
    # gauges only on the interior bonds of full dimension keep the host work bounded
    sites = product_state_mps([up if i % 2 == 0 else dn for i in range(n)], dims, rng)
    _, _, e = tn.mps_env_sweep(g32(sites), g32(inputs.xxz_mpo(n, delta)), store=False, prec=prec)
    e = e.cpu().numpy()
    ref = -delta * (n - 1) / 4
    assert abs(e[0] - ref) <= 2e-5 * n and abs(e[1] - ref) <= 2e-5 * n, (e, ref)


def test_env_sweep_chi1024_identity_channel_and_cuts():
    n, chi = 64, 1024
    raw = inputs.random_mps(n, 2, chi, 301)
    sites64 = [torch.tensor(x, device=DEV) for x in raw]
    tn.mps_left_canonicalize(sites64)
    psi = [s.float() for s in sites64]
    ls, rs, e = tn.mps_env_sweep(psi, g32(inputs.xxz_mpo(n, 0.5)), prec="split_bf16")
    torch.cuda.synchronize()
    for k in (1, 10, 32, 63):
        l0 = ls[k][:, 0, :].double()
        eye = torch.eye(l0.shape[0], dtype=torch.float64, device=DEV)
        assert float(torch.linalg.norm(l0 - eye) / math.sqrt(l0.shape[0])) < 1e-5
    e = e.cpu().numpy()
    cuts = [float((ls[k].double() * rs[k].double()).sum()) for k in (0, 16, 32, 48, 64)]
    for c in cuts:
        assert abs(c - e[0]) <= 1e-5 * max(1.0, abs(e[0])), (cuts, e)
