"""Host-side checks of bench.py's contract (no GPU): the one-GPU refusal and
the algorithmic flop count of the benchmark step."""
import os
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from paper_1905_01330_amd import inputs  # noqa: E402


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_sweep_flops_counts_each_contraction_once():
    """The step's flops equal the sum over sites of the four contractions'
    2 * (free sizes) * (contracted size) plus two MPO steps, counted here
    from the operands' shapes with numpy's own contraction cost."""
    n, chi = 10, 16
    dims = inputs.bond_dims(n, 2, chi)
    w = [1] + [5] * (n - 1) + [1]
    total = 0
    for k in range(n):
        da, db, wl, wr, d = dims[k], dims[k + 1], w[k], w[k + 1], 2
        shapes = [
            ("xua,asb->xusb", (da, wl, da), (da, d, db)),                  # L[a',u,a] . A[a,s,b]
            ("xtc,xtvb->cvb", (da, d, db), (da, d, wr, db)),               # A[a',t,b'] . T2[a',t,v,b]
            ("asb,cvb->ascv", (da, d, db), (db, wr, db)),                  # A[a,s,b] . R[b',v,b]
            ("xtc,uatc->xua", (da, d, db), (wl, da, d, db)),               # A[a',t,b'] . T2'[u,a,t,b']
            ("uvts,xusb->xtvb", (wl, wr, d, d), (da, wl, d, db)),          # W . T1 (left MPO step)
            ("uvts,asbv->uatb", (wl, wr, d, d), (da, d, db, wr)),          # W . T1' (right MPO step)
        ]
        for eq, sa, sb in shapes:
            _, info = np.einsum_path(eq, np.empty(sa), np.empty(sb), optimize=False)
            naive = [line for line in info.split("\n") if "Naive FLOP count" in line][0]
            total += float(naive.split(":")[1])
    assert bench.sweep_flops(dims, w) == total
