"""Benchmark: split-BF16 vs FP32 contraction throughput on one MI355X.

Workload (one "step"): the full left and right operator-environment sweep
of a chi = 1024 MPS (N = 64 sites, d = 2, bond dims min(chi, 2^k, 2^(N-k)))
with the XXZ chain MPO (bond 5, delta = 0.5); the MPS is random normal,
left-canonicalised in FP64 on the GPU and cast to FP32.  Every site runs
two contraction GEMMs and one MPO step per direction.  The reported value
is algorithmic TFLOP/s of the step in split-BF16 (six BF16 term products
per FP32 product, one FP32 accumulator); the FP32 path is timed beside it.

The roofline object is for the dominant kernel, the split-BF16 contraction
GEMM at the bulk-site shape (M = 5120, K = 1024, N = 2048: L_k[1024,5,1024]
against A_k[1024,2,1024]); its duration is measured with HIP events on the
stream it runs on, over replays of a HIP graph of that contraction alone
(`--mode tensordot` issues the same contraction eagerly, for profiling).  `cpu_baseline` times the FP64 oracle
on the whole step (both sweeps of the same chain) and compares every
environment and every headline output with the GPU path's.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--mode sweep|tensordot|rows|next|batched|canonicalize]

`--mode rows` times every row of the chain path against its roofline and `--mode next` the rows
beyond it (split_node, a two-site DMRG update, TTN and MERA networks), each with the oracle timed
beside it on a bounded sample.

`--mode batched` and `--mode canonicalize` run one row alone (the uneven batch,
all 512 chains or the first --chains, in --prec; the FP64 canonicalisation of
the chi = 1024 chain), for kernel-trace profiles.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK = {"bf16": 2516.6, "fp32": 157.3}  # dense TFLOP/s, MI355X published
N_SITES, CHI, W_BOND, DELTA, SEED = 64, 1024, 5, 0.5, 301
HEAD_M, HEAD_K, HEAD_N = 5120, 1024, 2048


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--mode", choices=["sweep", "tensordot", "rows", "next", "batched", "canonicalize", "profile",
                                       "mfma_rate"],
                    default="sweep")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU-baseline leg")
    ap.add_argument("--chains", type=int, default=512, help="--mode batched: first N chains of the uneven batch")
    ap.add_argument("--prec", default="fp32", help="--mode batched and profile: precision")
    ap.add_argument("--max-chi", type=int, default=0, help="--mode batched: only chains with chi <= this (0: all)")
    ap.add_argument("--tune", type=int, default=1, choices=[0, 1, 2],
                    help="--mode batched: tile autotuner level (0: the work estimate picks each step's tile)")
    ap.add_argument("--workload", choices=["chi1024", "chi256"], default="chi1024",
                    help="--mode profile: the XXZ N=64 chi=1024 sweep or the TFIM N=100 chi=256 sweep")
    ap.add_argument("--direction", choices=["left", "right", "both"], default="both", help="--mode profile")
    return ap.parse_args()


def sweep_flops(dims, w):
    """Algorithmic FLOPs of one left + right sweep (GEMMs and the MPO step)."""
    f = 0
    d = 2
    for k in range(len(dims) - 1):
        da, db, wl, wr = dims[k], dims[k + 1], w[k], w[k + 1]
        ws = 2 * da * db * (wl * d) * (d * wr)        # MPO step (each direction)
        f += 2 * (da * wl) * da * (d * db)            # left:  L . A over a
        f += 2 * db * (da * d) * (wr * db)            # left:  A . T2 over (a', t)
        f += 2 * (da * d) * db * (db * wr)            # right: A . R over b
        f += 2 * da * (d * db) * (wl * da)            # right: A . T2' over (t, b')
        f += 2 * ws
    return f


def gpu_inputs(torch, tn, inputs, n_sites=N_SITES, chi=CHI, seed=SEED, model="xxz"):
    """Random normal MPS, left-canonicalised in FP64 on the GPU and cast to
    FP32, and the chain's MPO (XXZ with delta = 0.5, or TFIM with J = g = 1)."""
    dev = torch.device("cuda:0")
    raw = inputs.random_mps(n_sites, 2, chi, seed)
    sites64 = [torch.tensor(x, device=dev) for x in raw]
    del raw
    tn.mps_left_canonicalize(sites64)
    psi = [s.float().contiguous() for s in sites64]
    del sites64
    ops = inputs.xxz_mpo(n_sites, DELTA) if model == "xxz" else inputs.tfim_mpo(n_sites)
    mpo = [torch.tensor(x, dtype=torch.float32, device=dev) for x in ops]
    torch.cuda.synchronize()
    return psi, mpo


def load_uneven_batch(torch, inputs, shapes):
    """All chains of the uneven batch, drawn on the host by a thread pool and
    copied to the device one chain (one buffer) at a time.  Returns the
    (psi, phi) site views per chain and the device buffers that own them."""
    import concurrent.futures as cf

    dev = torch.device("cuda:0")
    bufs, chains = [], []
    nthr = max(1, min(16, os.cpu_count() or 1))
    with cf.ThreadPoolExecutor(nthr) as ex:
        pending, nxt = {}, 0
        for i in range(len(shapes)):
            while nxt < len(shapes) and nxt < i + 2 * nthr:
                pending[nxt] = ex.submit(inputs.uneven_chain_flat, nxt, *shapes[nxt])
                nxt += 1
            flat, sh = pending.pop(i).result()
            dbuf = torch.from_numpy(flat).to(dev)
            del flat
            psi, phi, off = [], [], 0
            for part in (psi, phi):
                for s in sh:
                    cnt = s[0] * s[1] * s[2]
                    part.append(dbuf[off:off + cnt].view(*s))
                    off += cnt
            bufs.append(dbuf)
            chains.append((psi, phi))
    torch.cuda.synchronize()
    return chains, bufs


def copy_calibration(torch):
    """A plain 256 MiB device copy, three times: the reference kernel that
    calibrates the HBM byte counters of a profiled run."""
    src = torch.ones(64 << 20, device="cuda:0")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    return 2 * src.numel() * 4


def time_loop(torch, fn, steps, warmup):
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps  # ms


RATE_FLOPS = 256 * 8 * 5 * 6 * 32768 * 64   # issued flops of one rate measurement = T1's split-BF16 products


def product_rate(torch, tn, detail=False):
    """Issued-MFMA fraction of the split-BF16 product chains alone
    (tn_measure_split_mfma_rate at T1's issued flops), random then zero
    operand bits, after half a second of the same work to settle the clock."""
    out = torch.empty(131072, device="cuda:0")
    for _ in range(6000):
        tn.measure_split_mfma_rate(out, 64, False)
    torch.cuda.synchronize()
    res = {}
    for zero in (False, True):
        ms = time_loop(torch, lambda: tn.measure_split_mfma_rate(out, 64, zero), 200, 20)
        frac = round(RATE_FLOPS / (ms * 1e-3) / PEAK["bf16"] / 1e12, 4)
        res["zero" if zero else "random"] = {"us": round(1e3 * ms, 2), "issued_frac": frac} if detail else frac
    return res


HEAD_REPS = 20  # contractions per recorded graph in the headline loop


def headline_operands():
    """The bulk-site operands L[1024,5,1024] ~ N(0,1) and A[1024,2,1024] ~
    N(0,1)/sqrt(2048), drawn by numpy (seed 301) as float32."""
    import numpy as np

    rng = np.random.default_rng(SEED)
    L = rng.standard_normal((CHI, W_BOND, CHI)).astype(np.float32)
    A = (rng.standard_normal((CHI, 2, CHI)) / np.sqrt(2 * CHI)).astype(np.float32)
    return L, A


def headline(torch, tn, steps, warmup, graph=True, precs=("split_bf16", "fp32")):
    """The bulk-site contraction alone, per precision.

    With graph=True each timed step replays a HIP graph of HEAD_REPS
    back-to-back contractions, so the per-launch time is the kernel's and
    not the host's issue rate; without it the calls are issued eagerly
    (the form the kernel-trace profile records).  Returns the outputs too
    (host float64) for the oracle comparison of the CPU leg."""
    dev = torch.device("cuda:0")
    Lh, Ah = headline_operands()
    L, A = torch.tensor(Lh, device=dev), torch.tensor(Ah, device=dev)
    out = torch.empty((CHI, W_BOND, 2, CHI), device=dev)
    flops = 2.0 * HEAD_M * HEAD_K * HEAD_N
    res, outs = {}, {}
    for prec in precs:
        call = lambda: tn.contract_between(L, A, [2], [0], out=out, prec=prec)  # noqa: E731
        if graph:
            call()  # tile choice for this shape, outside the recording
            g = tn.Graph(lambda: [call() for _ in range(HEAD_REPS)])
            ms = time_loop(torch, g.replay, steps, warmup) / HEAD_REPS
        else:
            ms = time_loop(torch, call, steps, warmup)
        outs[prec] = out.cpu().double().numpy()
        res[prec] = {"ms": ms, "tflops": flops / ms / 1e9, "tile_config": tn.tune_last_choice()}
    return flops, res, outs


def traffic_for(tile_config):
    """HBM bytes per launch of the T1 split-BF16 GEMM from the committed PMC
    summary, if it was taken on the tile the tuner chose here and on the
    current source of that kernel."""
    p = os.path.join(ROOT, "profiles", "gemm_T1_split_bf16_traffic.json")
    if not os.path.exists(p):
        return None
    try:
        t = json.load(open(p))
        if t.get("tile_config") != tile_config:
            return None
        for name, sha in t.get("sources", {}).items():
            src = open(os.path.join(ROOT, "paper_1905_01330_amd", "csrc", name), "rb").read()
            if hashlib.sha1(src).hexdigest() != sha:
                return None
        return t.get("bytes_per_launch")
    except Exception:
        return None


def cpu_baseline_and_parity(torch, tn, inputs, head_outs):
    """The CPU-baseline leg: the FP64 oracle timed on the whole step (left
    and right sweeps of the same chi = 1024 chain), and the oracle's results
    compared with the GPU path's: every environment of the sweep in four
    precisions (on the oracle's own canonical MPS, rounded to FP32 and
    uploaded) and every output element of the headline contraction."""
    import numpy as np
    from threadpoolctl import threadpool_info

    import oracle

    dev = torch.device("cuda:0")
    can, _ = oracle.left_canonicalize(inputs.random_mps(N_SITES, 2, CHI, SEED))
    psi = [x.astype(np.float32).astype(np.float64) for x in can]
    del can
    mpo = inputs.xxz_mpo(N_SITES, DELTA)
    t0 = time.perf_counter()
    ls, rs, el, er = oracle.env_sweep(psi, mpo)
    dt = time.perf_counter() - t0
    dims = [1] + [x.shape[2] for x in psi]
    w = [1] + [x.shape[1] for x in mpo]
    threads = max([x.get("num_threads", 1) for x in threadpool_info()] or [1])
    base = {
        "value": sweep_flops(dims, w) / dt / 1e12,
        "unit": "TFLOP/s",
        "cores": int(threads),
        "kind": "oracle",
        "impl": "numpy FP64; a BLAS matmul is the product step of each tensordot",
        "sample": f"the whole step: left + right environment sweep of the chi=1024, N=64 XXZ chain, FP64, "
                  f"{dt:.1f} s on {int(threads)} BLAS threads",
        "seconds": dt,
    }
    gpsi = [torch.tensor(x, dtype=torch.float32, device=dev) for x in psi]
    gmpo = [torch.tensor(x, dtype=torch.float32, device=dev) for x in mpo]
    env_err, energy_err = {}, {}
    for prec in ("split_bf16", "fp32", "bf16", "split_bf16_3p"):
        sw = tn.EnvSweep(gpsi, gmpo, left=True, right=True, store=True, prec=prec).run()
        torch.cuda.synchronize()
        e = 0.0
        for k in range(1, N_SITES):
            for got, ref in ((sw.L[k], ls[k]), (sw.R[k], rs[k])):
                g = got.cpu().double().numpy()
                e = max(e, float(np.linalg.norm(g - ref) / np.linalg.norm(ref)))
        env_err[prec] = e
        en = sw.energy.cpu().numpy()
        energy_err[prec] = max(abs(en[0] - el) / abs(el), abs(en[1] - er) / abs(er))
        del sw
    Lh, Ah = headline_operands()
    ref = oracle.tensordot(Lh, Ah, [2], [0])
    head_err = {p: float(np.linalg.norm(o - ref) / np.linalg.norm(ref)) for p, o in head_outs.items()}
    parity = {
        "oracle": "FP64 numpy oracle, whole outputs (every L_k, R_k with 0 < k < N; every element of T1)",
        "env_max_rel_err": env_err,
        "energy_rel_err": energy_err,
        "headline_rel_err": head_err,
    }
    return base, parity


# ---------------------------------------------------------------------------
# --mode rows: every step of the path on its own, against its roofline, with
# the oracle timed beside it on a bounded sample

PEAK_ROWS = {"hbm": (8000.0, "GB/s"), "bf16": (PEAK["bf16"], "TFLOP/s"), "fp32": (PEAK["fp32"], "TFLOP/s"),
             "fp64": (78.6, "TFLOP/s")}


def _gtime(torch, tn, fn, reps=10, steps=3, warmup=1):
    """ms per call of fn (launch-only calls), over replays of a graph of `reps` calls."""
    fn()
    torch.cuda.synchronize()
    g = tn.Graph(lambda: [fn() for _ in range(reps)])
    return time_loop(torch, g.replay, steps, warmup) / reps


def _ctime(fn, min_s=1.0):
    """seconds per call of a host (oracle) function, repeated for at least min_s."""
    n, t0 = 0, time.perf_counter()
    while True:
        fn()
        n += 1
        dt = time.perf_counter() - t0
        if dt >= min_s:
            return dt / n


def _row(rid, what, workload, work, ms, kind, cpu_work, cpu_s, sample, extra=None):
    """work / cpu_work: bytes (kind 'hbm') or flops per call."""
    peak, unit = PEAK_ROWS[kind]
    scale = 1e9 if unit == "GB/s" else 1e12
    val = work / (ms * 1e-3) / scale
    print(f"row {rid} done: {ms:.4f} ms", file=sys.stderr, flush=True)
    r = {"row": rid, "what": what, "workload": workload, "ms": round(ms, 4),
         "roofline": {"bound": "hbm" if kind == "hbm" else "mfma", "achieved": round(val, 3), "peak": peak,
                      "unit": unit, "frac": round(val / peak, 4)},
         "cpu_oracle": {"value": round(cpu_work / cpu_s / scale, 4), "unit": unit, "sample": sample,
                        "seconds_per_call": round(cpu_s, 4)}}
    if extra:
        r.update(extra)
    return r


def rows(torch, tn, inputs):
    import numpy as np

    import oracle

    dev = torch.device("cuda:0")
    gen = torch.Generator(device=dev).manual_seed(SEED)
    rn = lambda *shape: torch.randn(shape, device=dev, generator=gen)  # noqa: E731
    out = []
    tn.tune_set_level(1)

    # a1-a4: the two headline tensordots of a bulk site (T1, T3 with its permuted
    # store), on the headline's operands and timed as the headline is
    Lnp, Anp = headline_operands()
    L, A = torch.tensor(Lnp, device=dev), torch.tensor(Anp, device=dev)
    T2 = torch.tensor(np.random.default_rng(SEED + 1).standard_normal((CHI, 2, W_BOND, CHI)).astype(np.float32),
                      device=dev)
    o1 = torch.empty((CHI, W_BOND, 2, CHI), device=dev)
    Lout = torch.empty((CHI, W_BOND, CHI), device=dev)
    o3 = Lout.permute(1, 2, 0)     # T2 . A -> [v, b, b'] stored into L[b', v, b]
    fl = 2.0 * HEAD_M * HEAD_K * HEAD_N
    Lh, Ah, T2h = (x.cpu().double().numpy() for x in (L, A, T2))
    for prec, kind in (("split_bf16", "bf16"), ("fp32", "fp32")):
        ms1 = _gtime(torch, tn, lambda: tn.contract_between(L, A, [2], [0], out=o1, prec=prec), reps=HEAD_REPS,
                     steps=5, warmup=2)
        tile1 = tn.tune_last_choice()
        ms3 = _gtime(torch, tn, lambda: tn.contract_between(T2, A, [0, 1], [0, 1], out=o3, prec=prec),
                     reps=HEAD_REPS, steps=5, warmup=2)
        tile3 = tn.tune_last_choice()
        c1 = _ctime(lambda: oracle.contract_between(Lh[:64], Ah, [(2, 0)]))
        c3 = _ctime(lambda: oracle.contract_between(T2h, Ah[:, :, :64], [(0, 0), (1, 1)]))
        w1 = "L[1024,5,1024] . A[1024,2,1024] over (2,0): M=5120 K=1024 N=2048"
        w3 = "T2[1024,2,5,1024] . A[1024,2,1024] over ((0,1),(0,1)), stored permuted into L[1024,5,1024]"
        extra = {"precision": prec, "tile_config": tile1}
        if prec == "split_bf16":
            extra["issued_mfma_frac"] = round(6 * fl / (ms1 * 1e-3) / 1e12 / PEAK["bf16"], 4)
        out.append(_row("a1-a4 T1", "tensordot (plan, fused gather, GEMM, epilogue)", w1, fl, ms1, kind,
                        2.0 * 64 * 5 * 1024 * 2048, c1, "first 64 rows of L", extra))
        extra = {"precision": prec, "tile_config": tile3}
        out.append(_row("a1-a4 T3", "tensordot with a permuted output", w3, fl, ms3, kind,
                        2.0 * 64 * 2048 * 5120, c3, "first 64 columns of A", extra))
    del L, A, T2, o1, Lout, Lh, Ah, T2h

    # a5: rank-0 and rank-1 results
    n = 1 << 28
    x, y = rn(n), rn(n)
    ms = _gtime(torch, tn, lambda: tn.contract_between(x, y, [0], [0]))
    xs, ys = x[: 1 << 24].cpu().double().numpy(), y[: 1 << 24].cpu().double().numpy()
    c = _ctime(lambda: oracle.contract_between(xs, ys, [(0, 0)]))
    out.append(_row("a5 dot", "rank-0 result (FP64 accumulation)", "x[2^28] . y[2^28]", 8.0 * n, ms, "hbm",
                    16.0 * (1 << 24), c, "first 2^24 elements (FP64)"))
    del x, y
    m = 16384
    M_, v = rn(m, m), rn(m)
    mv = torch.empty(m, device=dev)
    ms = _gtime(torch, tn, lambda: tn.contract_between(M_, v, [1], [0], out=mv))
    Ms, vs = M_[:1024].cpu().double().numpy(), v.cpu().double().numpy()
    c = _ctime(lambda: oracle.contract_between(Ms, vs, [(1, 0)]))
    out.append(_row("a5 matvec", "rank-1 result", "M[16384,16384] . v[16384]", 4.0 * (m * m + 2 * m), ms, "hbm",
                    8.0 * 1024 * m, c, "first 1024 rows (FP64)"))
    del M_, v, mv

    # a6: trace edge over the two leading axes of A[64, 64, 2^18] (reads 64 contiguous rows)
    D, X = 64, 1 << 18
    T = rn(D, D, X)
    tr = torch.empty(X, device=dev)
    ms = _gtime(torch, tn, lambda: tn.trace_edge(T, 0, 1, out=tr))
    Ts = T[:, :, : 1 << 14].cpu().double().numpy()
    c = _ctime(lambda: oracle.trace_edge(Ts, 0, 1))
    out.append(_row("a6", "trace edge", "A[64, 64, 2^18], trace over axes 0 and 1", 4.0 * (D * X + X), ms, "hbm",
                    8.0 * (D * (1 << 14) + (1 << 14)), c, "A[:, :, :2^14] (FP64)"))
    del T, tr

    # a7: outer product (write-bound)
    a, b = rn(8192), rn(32768)
    op = torch.empty((8192, 32768), device=dev)
    ms = _gtime(torch, tn, lambda: tn.outer_product(a, b, out=op))
    a_s, b_s = a.cpu().double().numpy(), b[:4096].cpu().double().numpy()
    c = _ctime(lambda: oracle.outer_product(a_s, b_s))
    out.append(_row("a7", "outer product", "a[8192] (x) b[32768]", 4.0 * (8192 + 32768 + 8192 * 32768), ms, "hbm",
                    8.0 * (8192 + 4096 + 8192 * 4096), c, "b[:4096] (FP64)"))
    del a, b, op

    # a8: ncon network = one environment step (L, A, W, A) with a given order
    psi, mpo = gpu_inputs(torch, tn, inputs)
    k = N_SITES // 2
    Lk = rn(CHI, W_BOND, CHI) / CHI
    tens = [Lk, psi[k], mpo[k], psi[k]]
    labels = [[1, 2, 3], [3, 4, -3], [2, -2, 5, 4], [1, 5, -1]]
    order = [3, 2, 4, 1, 5]
    netout = torch.empty((CHI, W_BOND, CHI), device=dev)
    for prec, kind in (("split_bf16", "bf16"), ("fp32", "fp32")):
        ms = _gtime(torch, tn, lambda: tn.contract_network(tens, labels, order=order, out=netout, prec=prec), reps=4)
        nfl = 2.0 * (CHI * W_BOND) * CHI * (2 * CHI) + 2.0 * (CHI * CHI * 2) * (W_BOND * 2) * (W_BOND * 2) / 2 \
            + 2.0 * CHI * (CHI * 2) * (W_BOND * CHI)
        hs = [t.cpu().double().numpy() for t in tens]
        hs[0], hs[3] = hs[0][:128], hs[3][:128]
        c = _ctime(lambda: oracle.contract_network(hs, labels, order=order))
        cfl = nfl * 128 / CHI
        out.append(_row("a8", "ncon network driver", "L[1024,5,1024] A[1024,2,1024] W[5,5,2,2] A[1024,2,1024], "
                        "order 3,2,4,1,5", nfl, ms, kind, cfl, c, "bra bond cut to 128 (FP64)", {"precision": prec}))

    # a9: MPS inner product of the chi = 1024 chain with itself
    dims = [1] + [int(t.shape[2]) for t in psi]
    ifl = sum(4.0 * dims[i] ** 2 * dims[i + 1] + 4.0 * dims[i] * dims[i + 1] ** 2 for i in range(N_SITES))
    small = [x.astype(np.float64) for x in inputs.random_mps(N_SITES, 2, 128, SEED)]
    sd = [1] + [x.shape[2] for x in small]
    sfl = sum(4.0 * sd[i] ** 2 * sd[i + 1] + 4.0 * sd[i] * sd[i + 1] ** 2 for i in range(N_SITES))
    c = _ctime(lambda: oracle.mps_inner(small, small))
    for prec, kind in (("split_bf16", "bf16"), ("fp32", "fp32")):
        ms = _gtime(torch, tn, lambda: tn.mps_inner(psi, psi, prec=prec), reps=4)
        out.append(_row("a9", "MPS inner product", "<psi|psi>, N=64, chi=1024", ifl, ms, kind, sfl, c,
                        "full chain at chi=128 (FP64)", {"precision": prec}))

    # a10: the environment sweep (the bench step)
    dw = [1] + [int(t.shape[1]) for t in mpo]
    sfl10 = sweep_flops(dims, dw)
    sw = tn.EnvSweep(psi, mpo, left=True, right=True, store=True, prec="split_bf16")
    ms = _gtime(torch, tn, sw.run, reps=1, steps=3)
    l = np.ones((1, 1, 1))
    sites = [t.cpu().double().numpy() for t in psi[20:22]]
    mp = [t.cpu().double().numpy() for t in mpo[20:22]]
    l = np.random.default_rng(0).standard_normal((dims[20], dw[20], dims[20]))
    c = _ctime(lambda: oracle.env_left_step(l, sites[0], mp[0]))
    cfl = 2.0 * (dims[20] * dw[20]) * dims[20] * (2 * dims[21]) + 2.0 * dims[21] * (dims[20] * 2) * (dw[21] * dims[21])
    out.append(_row("a10", "environment sweep, left + right", "XXZ, N=64, chi=1024, MPO bond 5", sfl10, ms, "bf16",
                    cfl, c, "one bulk left step (FP64)", {"precision": "split_bf16"}))
    del sw

    # a10 at chi = 256: the TFIM sweep, N = 100 (latency-bound sites)
    del psi
    psi2, mpo2 = gpu_inputs(torch, tn, inputs, n_sites=100, chi=256, seed=201, model="tfim")
    d2 = [1] + [int(t.shape[2]) for t in psi2]
    w2 = [1] + [int(t.shape[1]) for t in mpo2]
    fl2 = sweep_flops(d2, w2)
    for prec, kind in (("split_bf16", "bf16"), ("fp32", "fp32")):
        sw2 = tn.EnvSweep(psi2, mpo2, left=True, right=True, store=True, prec=prec)
        ms = _gtime(torch, tn, sw2.run, reps=2, steps=5, warmup=2)
        sites = [t.cpu().double().numpy() for t in psi2[50:51]]
        l2 = np.random.default_rng(0).standard_normal((d2[50], w2[50], d2[50]))
        mp2 = mpo2[50].cpu().double().numpy()
        c = _ctime(lambda: oracle.env_left_step(l2, sites[0], mp2))
        cfl = 2.0 * (d2[50] * w2[50]) * d2[50] * (2 * d2[51]) + 2.0 * d2[51] * (d2[50] * 2) * (w2[51] * d2[51])
        out.append(_row("a10 chi=256", "environment sweep, left + right", "TFIM, N=100, chi=256, MPO bond 3", fl2, ms,
                        kind, cfl, c, "one bulk left step (FP64)", {"precision": prec}))
        del sw2
    del psi2, mpo2

    # a12: uneven batch, all 512 chains of the workload in one call
    shapes = inputs.uneven_chain_shapes()
    chains, keep = load_uneven_batch(torch, inputs, shapes)
    bfl = 0.0
    for nn, chi in shapes:
        d_ = inputs.bond_dims(nn, 2, chi)
        bfl += sum(4.0 * d_[j] ** 2 * d_[j + 1] + 4.0 * d_[j] * d_[j + 1] ** 2 for j in range(nn))
    cheap = sorted(range(len(shapes)), key=lambda i: shapes[i][0] * shapes[i][1] ** 3)[:4]
    host = [inputs.uneven_chain(i, *shapes[i]) for i in cheap]
    host = [([x.astype(np.float64) for x in p], [x.astype(np.float64) for x in q]) for p, q in host]
    hfl = 0.0
    for p, q in host:
        d_ = [1] + [x.shape[2] for x in p]
        hfl += sum(4.0 * d_[j] ** 2 * d_[j + 1] + 4.0 * d_[j] * d_[j + 1] ** 2 for j in range(len(p)))
    c = _ctime(lambda: [oracle.mps_inner(p, q) for p, q in host])
    for prec, kind in (("fp32", "fp32"), ("split_bf16", "bf16")):
        bi = tn.BatchedInner(chains, prec)
        ms = _gtime(torch, tn, bi.run, reps=1, steps=3, warmup=1)
        out.append(_row("a12", "uneven batched inner products, one call", "all 512 chains (N ~ U{8..256}, "
                        "chi ~ U{8..512}, 84 GB)", bfl, ms, kind, hfl, c, "the 4 cheapest chains (FP64)",
                        {"precision": prec}))
        del bi
    del chains, keep
    torch.cuda.empty_cache()

    # a11, a13: classifier forward (cfg4a) and training step (cfg5)
    for tag, (n_, chi, B, seed) in (("cfg4a", (784, 64, 4096, 401)), ("cfg5", (784, 128, 1024, 501))):
        c_ = n_ // 2
        sites = [torch.tensor(s, dtype=torch.float32, device=dev) for s in inputs.classifier_sites(n_, chi, 10, c_, seed)]
        pix = torch.tensor(inputs.images(B, n_, seed + 1), dtype=torch.float32, device=dev)
        lab = torch.tensor(inputs.labels(B, 10, seed + 2), device=dev)
        model = tn.MPSClassifier(n_, c_, 10, chi, B, ckpt_every=28, prec="split_bf16")
        ffl = 2.0 * B * (2 * chi) * chi * (n_ - 1) + 2.0 * B * (2 * chi) * (10 * chi)
        hs = [s.cpu().double().numpy() for s in sites]
        hp = pix[:4].cpu().double().numpy()
        c = _ctime(lambda: oracle.classifier_forward(hs, c_, hp))
        ms = _gtime(torch, tn, lambda: model.forward(sites, pix), reps=2)
        out.append(_row("a11", "classifier forward", f"{tag}: N=784, chi={chi}, batch {B}", ffl, ms, "fp64",
                        ffl * 4 / B, c, "4 samples (FP64)", {"note": "chains on FP64 matrix cores"}))
        if tag == "cfg5":
            logits = model.forward(sites, pix)
            _, dlog = tn.softmax_xent(logits, lab)
            dsites = [torch.empty_like(s) for s in sites]

            def step():
                model.forward(sites, pix, logits)
                model.backward(sites, pix, dlog, dsites)

            ms = _gtime(torch, tn, step, reps=1)
            c = _ctime(lambda: oracle.classifier_loss_and_grad(hs, c_, hp, lab[:4].cpu().numpy()))
            out.append(_row("a13", "classifier training step (forward + adjoint + weight gradients)",
                            f"{tag}: N=784, chi={chi}, batch {B}, checkpoints every 28 sites", 3 * ffl, ms, "fp64",
                            3 * ffl * 4 / B, c, "4 samples (FP64)",
                            {"note": "algorithmic = 3 x forward; the checkpoint recompute is extra work"}))
        del model, sites, pix

    # a14: FP64 Householder canonicalisation of the chi = 1024 chain
    raw = [torch.tensor(x, device=dev) for x in inputs.random_mps(N_SITES, 2, CHI, SEED)]
    qfl = 0.0
    for i in range(N_SITES):
        mm, nn_ = dims[i] * 2, dims[i + 1]
        qfl += 4.0 * mm * nn_ * nn_ - 4.0 * nn_ ** 3 / 3 + (2.0 * nn_ * nn_ * 2 * dims[i + 2] if i + 1 < N_SITES else 0)
    work = [x.clone() for x in raw]

    def canon():
        for w_, r_ in zip(work, raw):
            w_.copy_(r_)
        tn.mps_left_canonicalize(work)

    canon()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    canon()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3
    hs = [x.astype(np.float64) for x in inputs.random_mps(N_SITES, 2, 128, SEED)]
    d2 = [1] + [x.shape[2] for x in hs]
    hfl = sum(4.0 * d2[i] * 2 * d2[i + 1] ** 2 - 4.0 * d2[i + 1] ** 3 / 3 for i in range(N_SITES))
    c = _ctime(lambda: oracle.left_canonicalize(hs))
    out.append(_row("a14", "FP64 Householder canonicalisation (support)", "N=64, chi=1024 random MPS", qfl, ms,
                    "fp64", hfl, c, "full chain at chi=128 (LAPACK QR, FP64)",
                    {"note": "host-timed (includes the copy of the raw chain)"}))
    return out


def next_rows(torch, tn, inputs):
    """Rows beyond the chain networks: node splitting (the paper's 1000 x 1000
    truncation example), one two-site DMRG update at chi = 256, and the
    TTN / MERA expectation networks, each against its roofline with the
    oracle timed beside it on a bounded sample."""
    import numpy as np

    import oracle
    from paper_1905_01330_amd import networks

    dev = torch.device("cuda:0")
    out = []
    rng = np.random.default_rng(SEED)

    # split_node of a 1000 x 1000 node (FP64), max_singular_values = 5
    n = 1000
    q1 = np.linalg.qr(rng.standard_normal((n, n)))[0]
    q2 = np.linalg.qr(rng.standard_normal((n, n)))[0]
    a = (q1 * np.exp(-np.arange(n) / 40.0)[None, :]) @ q2.T
    ga = torch.tensor(a, device=dev)
    tn.split_node(ga, [0], [1], max_singular_values=5)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    reps = 3
    for _ in range(reps):
        tn.split_node(ga, [0], [1], max_singular_values=5)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) / reps * 1e3
    svd_flops = 4.0 * n * n * n + 8.0 * n * n * n + 9.0 * n ** 3   # thin SVD with both factors (Golub and Van Loan)
    c = _ctime(lambda: oracle.split_node(a, 1, max_singular_values=5))
    out.append(_row("n1", "split_node, FP64 one-sided block Jacobi SVD + truncation", "1000 x 1000 node, "
                    "max_singular_values=5 (Appendix A example)", svd_flops, ms, "fp64", svd_flops, c,
                    "the same node (numpy LAPACK SVD)", {"note": "host-timed; synchronising call"}))

    # complex contraction at the bulk-site shape: L[1024,5,1024] . conj(A[1024,2,1024]) over (2,0)
    lc = (rng.standard_normal((1024, 5, 1024)) + 1j * rng.standard_normal((1024, 5, 1024))).astype(np.complex64)
    ac = ((rng.standard_normal((1024, 2, 1024)) + 1j * rng.standard_normal((1024, 2, 1024))) /
          np.sqrt(4096)).astype(np.complex64)
    glc, gac = torch.tensor(lc, device=dev), torch.tensor(ac, device=dev)
    cfl = 8.0 * 5120 * 2048 * 1024          # four real products and four additions per complex term
    lch = lc[:64].astype(np.complex128)
    ach = ac.astype(np.complex128)
    cc = _ctime(lambda: oracle.tensordot_c(lch, ach, [2], [0], False, True))
    for prec, kind in (("split_bf16", "bf16"), ("fp32", "fp32")):
        ms = _gtime(torch, tn, lambda: tn.contract_between(glc, gac, [2], [0], prec=prec, conj_b=True), reps=5)
        out.append(_row("n2", "complex tensordot, conjugated right operand (expansion + one real contraction)",
                        "L[1024,5,1024] . conj(A[1024,2,1024]) over (2,0), complex64", cfl, ms, kind,
                        cfl * 64 / 1024, cc, "first 64 rows of L (complex FP64)", {"precision": prec}))
    del glc, gac, lc, ac, lch, ach

    # one two-site DMRG update at chi = 256 (TFIM, bulk sites of the N = 100 chain)
    psi, mpo = gpu_inputs(torch, tn, inputs, n_sites=100, chi=256, seed=201, model="tfim")
    ls, _, _ = tn.mps_env_sweep(psi, mpo, left=True, right=False, store=True)
    _, rs, _ = tn.mps_env_sweep(psi, mpo, left=False, right=True, store=True)
    k = 50
    theta0 = tn.contract_between(psi[k], psi[k + 1], [2], [0]).contiguous()
    shapes, labels = [tuple(x.shape) for x in (ls[k], theta0, mpo[k], mpo[k + 1], rs[k + 2])], \
        [[-1, 1, 2], [2, 3, 4, 5], [1, 6, -2, 3], [6, 7, -3, 4], [-4, 7, 5]]
    _, mv_flops = tn.network_order([ls[k], theta0, mpo[k], mpo[k + 1], rs[k + 2]], labels, "greedy")
    for prec, kind in (("split_bf16", "bf16"), ("fp32", "fp32")):
        th = theta0.clone()
        tn.dmrg_two_site_update(ls[k], rs[k + 2], mpo[k], mpo[k + 1], th, chi_max=256, krylov=24, restarts=2,
                                prec=prec)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        th = theta0.clone()
        out2, _, _, _ = tn.dmrg_two_site_update(ls[k], rs[k + 2], mpo[k], mpo[k + 1], th, chi_max=256, krylov=24,
                                                restarts=2, prec=prec)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3
        n_mv = 24 * 2 + 1
        fl = mv_flops * n_mv
        lh = ls[k][:64, :, :64].cpu().double().numpy()
        rh = rs[k + 2][:64, :, :64].cpu().double().numpy()
        th_h = np.random.default_rng(0).standard_normal((64, 2, 2, 64))
        w1, w2 = mpo[k].cpu().double().numpy(), mpo[k + 1].cpu().double().numpy()
        cc = _ctime(lambda: oracle.heff_apply(lh, rh, w1, w2, th_h))
        cfl = mv_flops * (64 / 256) ** 3
        out.append(_row("n3", "two-site DMRG update: 49 H_eff mat-vecs (Lanczos, 24 vectors, 2 restarts) + split",
                        "TFIM N=100, chi=256, sites 50-51", fl, ms, kind, cfl, cc,
                        "one H_eff mat-vec at chi=64 (FP64)",
                        {"precision": prec, "energy": float(out2[0].cpu()), "residual": float(out2[1].cpu()),
                         "note": "host-timed, includes the synchronising split; flops count the mat-vecs only"}))
    del psi, mpo, ls, rs

    # TTN (N = 256, chi = 64) and binary MERA (N = 16, chi = 16): <Z Z> on two middle sites
    zz = np.diag([1.0, -1.0])
    for name, nn, chi, mera, csample in (("n4 TTN", 256, 64, False, (64, 32)), ("n4 MERA", 16, 16, True, (16, 4))):
        mid = nn // 2 - 1
        shapes, labels, src = networks.expectation(nn, 2, chi, (mid, mid + 1), mera)
        net, _ = networks.tree_state(nn, 2, chi, mera)
        g = np.random.default_rng(7)
        state = [torch.tensor(g.standard_normal(s) / np.sqrt(s[0] * s[1]), dtype=torch.float32, device=dev)
                 for s in net.shapes]
        zt = torch.tensor(zz, dtype=torch.float32, device=dev)
        nodes = [state[i] if i >= 0 else zt for i in src]
        order, fl = tn.network_order(nodes, labels, "greedy")
        sh, sl, ss = networks.expectation(csample[0], 2, csample[1], (3, 4), mera)
        snet, _ = networks.tree_state(csample[0], 2, csample[1], mera)
        hs = [g.standard_normal(s) / np.sqrt(s[0] * s[1]) for s in snet.shapes]
        hn = [hs[i] if i >= 0 else zz for i in ss]
        horder, hfl = tn.network_order([torch.empty(s) for s in sh], sl, "greedy")
        c = _ctime(lambda: oracle.contract_network(hn, sl, horder))
        for prec, kind in (("split_bf16", "bf16"), ("fp32", "fp32")):
            ms = _gtime(torch, tn, lambda: tn.contract_network(nodes, labels, order=order, prec=prec), reps=2)
            out.append(_row(name, f"<psi|Z Z|psi> network ({len(nodes)} nodes, greedy order)",
                            f"N={nn}, chi={chi}, d=2", fl, ms, kind, hfl, c,
                            f"N={csample[0]}, chi={csample[1]} (FP64, the same order search)", {"precision": prec}))
    return out


def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py measures one GPU only (--gpus {a.gpus} requested); the sweep would shard the "
              "environment bond across GPUs with a reduce-scatter per site, which is not built.", file=sys.stderr)
        sys.exit(2)
    import torch

    import paper_1905_01330_amd as tn
    from paper_1905_01330_amd import inputs

    if a.mode in ("rows", "next"):
        res = rows(torch, tn, inputs) if a.mode == "rows" else next_rows(torch, tn, inputs)
        for r in res:
            print(json.dumps(r))
        print("| row | workload | ms | achieved | roofline | frac | oracle (sample) |")
        print("|---|---|---|---|---|---|---|")
        for r in res:
            f, o = r["roofline"], r["cpu_oracle"]
            p = f" ({r['precision']})" if "precision" in r else ""
            print(f"| {r['row']}{p} | {r['workload']} | {r['ms']:.3f} | {f['achieved']:.3g} {f['unit']} | "
                  f"{f['bound']} {f['peak']:g} | {f['frac']:.4f} | {o['value']:.3g} {o['unit']} ({o['sample']}) |")
        return
    if a.mode == "batched":
        shapes = inputs.uneven_chain_shapes()
        if a.chains < len(shapes):
            shapes = shapes[:a.chains]
        if a.max_chi:
            shapes = [s for s in shapes if s[1] <= a.max_chi]
        chains, keep = load_uneven_batch(torch, inputs, shapes)
        if a.tune == 2:
            tn.tune(None, 2)
        else:
            tn.tune_set_level(a.tune)
        bi = tn.BatchedInner(chains, a.prec)
        ms = time_loop(torch, bi.run, a.steps, a.warmup)   # the first warm-up call times the step tiles
        del bi, chains, keep
        print(json.dumps({"mode": "batched", "chains": len(shapes), "precision": a.prec, "tune": a.tune,
                          "ms_per_call": round(ms, 4), "copy_bytes": copy_calibration(torch)}))
        return
    if a.mode == "profile":
        # one sweep configuration in one or both directions, for kernel traces
        # and HBM counters of its kernels alone
        tn.tune_set_level(1)
        if a.workload == "chi1024":
            psi, mpo = gpu_inputs(torch, tn, inputs)
        else:
            psi, mpo = gpu_inputs(torch, tn, inputs, n_sites=100, chi=256, seed=201, model="tfim")
        sw = tn.EnvSweep(psi, mpo, left=a.direction != "right", right=a.direction != "left", store=True,
                         prec=a.prec)
        ms = time_loop(torch, sw.run, a.steps, a.warmup)
        del sw, psi, mpo
        print(json.dumps({"mode": "profile", "workload": a.workload, "direction": a.direction, "precision": a.prec,
                          "ms_per_call": round(ms, 4), "copy_bytes": copy_calibration(torch)}))
        return
    if a.mode == "canonicalize":
        dev = torch.device("cuda:0")
        raw = [torch.tensor(x, device=dev) for x in inputs.random_mps(N_SITES, 2, CHI, SEED)]
        times = []
        for it in range(a.warmup + a.steps):
            sites = [x.clone() for x in raw]
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            tn.mps_left_canonicalize(sites)
            torch.cuda.synchronize()
            if it >= a.warmup:
                times.append(time.perf_counter() - t0)
        print(json.dumps({"mode": "canonicalize", "n_sites": N_SITES, "chi": CHI,
                          "ms_per_call": round(1e3 * sum(times) / max(len(times), 1), 3)}))
        return
    if a.mode == "mfma_rate":
        print(json.dumps({"mode": "mfma_rate", "issued_flops": RATE_FLOPS, **product_rate(torch, tn, detail=True)}))
        return
    if a.mode == "tensordot":
        tn.tune_set_level(1)
        flops, res, _ = headline(torch, tn, a.steps, a.warmup, graph=False)
        print(json.dumps({"mode": "tensordot", "flops": flops, "copy_bytes": copy_calibration(torch), **res}))
        return

    tn.tune_set_level(1)   # time the tile candidates once per contraction shape (during warm-up)
    psi, mpo = gpu_inputs(torch, tn, inputs)
    dims = [1] + [int(x.shape[2]) for x in psi]
    w = [1] + [int(x.shape[1]) for x in mpo]
    flops = sweep_flops(dims, w)

    sweeps = {p: tn.EnvSweep(psi, mpo, left=True, right=True, store=True, prec=p) for p in ("split_bf16", "fp32")}
    ms = {}
    for p, s in sweeps.items():
        ms[p] = time_loop(torch, s.run, a.steps, a.warmup)
    # the same sweep recorded once as a HIP graph and replayed
    gsweep = tn.Graph(sweeps["split_bf16"].run)
    ms_graph = time_loop(torch, gsweep.replay, a.steps, a.warmup)
    energy = float(sweeps["split_bf16"].energy[0].item())
    e32 = float(sweeps["fp32"].energy[0].item())

    hflops, head, head_outs = headline(torch, tn, max(a.steps, 5), 2,
                                       precs=("split_bf16", "fp32", "bf16", "split_bf16_3p"))
    x6 = head["split_bf16"]
    achieved = x6["tflops"]
    traffic = traffic_for(x6["tile_config"])
    rate = product_rate(torch, tn)

    value = flops / (ms["split_bf16"] * 1e-3) / 1e12
    line = {
        "metric": "TFLOP/s & % MFMA peak: split-BF16 vs FP32 tensordot at rel err <=1e-6",
        "value": round(value, 3),
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(ms["split_bf16"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16x6-f32acc",
        "data": "synthetic",
        "config": {
            "workload": "XXZ MPS-MPO-MPS left+right environment sweep, N=64, d=2, chi=1024, MPO bond 5, "
                        "delta=0.5, random MPS (seed 301) left-canonicalised in FP64",
            "n_sites": N_SITES, "chi": CHI, "mpo_bond": W_BOND, "precision": "split_bf16",
        },
        "roofline": {
            "bound": "mfma",
            "achieved": round(achieved, 3),
            "peak": PEAK["bf16"],
            "unit": "TFLOP/s",
            "frac": round(achieved / PEAK["bf16"], 5),
            "traffic": traffic,
            "kernel": "split-BF16 contraction GEMM, M=5120 K=1024 N=2048 (bulk site, L_k . A_k)",
            "issued_mfma_frac": round(6 * achieved / PEAK["bf16"], 4),
            "launch_ms": round(x6["ms"], 5),
            "tile_config": x6["tile_config"],
            # the same six-product chains with register operands (no loads,
            # no LDS), random and zero operand bits: what the chip sustains
            "product_rate_issued_frac": rate,
        },
        "fp32_path": {
            "value": round(flops / (ms["fp32"] * 1e-3) / 1e12, 3),
            "ms_per_step": round(ms["fp32"], 4),
            "headline_tflops": round(head["fp32"]["tflops"], 3),
            "headline_frac_of_fp32_peak": round(head["fp32"]["tflops"] / PEAK["fp32"], 4),
        },
        "speedup_split_bf16_vs_fp32": round(ms["fp32"] / ms["split_bf16"], 3),
        "headline_tflops": {p: round(r["tflops"], 3) for p, r in head.items()},
        "energy": {"split_bf16": energy, "fp32": e32},
        "flops_per_step": flops,
        "graph_replay": {"value": round(flops / (ms_graph * 1e-3) / 1e12, 3), "ms_per_step": round(ms_graph, 4)},
    }
    del sweeps, gsweep
    torch.cuda.empty_cache()
    if not a.no_cpu:
        line["cpu_baseline"], line["parity"] = cpu_baseline_and_parity(torch, tn, inputs, head_outs)
    print(json.dumps(line))


if __name__ == "__main__":
    main()
