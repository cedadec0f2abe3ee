"""Oracle: bit-level model of the BF16 operand rounding and the 3-term split.

Test infrastructure only (see the package docstring).

bf16(x) rounds an FP32 value to the nearest value with an 8-bit significand
(round half to even).  The split writes x = x0 + x1 + x2 with
x0 = bf16(x), x1 = bf16(x - x0), x2 = bf16(x - x0 - x1); for normal FP32
inputs the three terms reproduce x exactly.  The compensated product keeps
the six term products x_i * y_j with i + j <= 2 (Henry, Tang and Heinecke,
ARITH 2019).
"""
from __future__ import annotations

import numpy as np


def bf16_round(x):
    """Round FP32 values to BF16 (returned as FP32), nearest-even on the bit pattern."""
    x = np.asarray(x, dtype=np.float32)
    u = x.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) & 0xFFFF0000).astype(np.uint32)
    out = r.view(np.float32)
    return np.where(np.isfinite(x), out, x)


def split3(x):
    x = np.asarray(x, dtype=np.float32)
    x0 = bf16_round(x)
    r1 = (x - x0).astype(np.float32)
    x1 = bf16_round(r1)
    x2 = bf16_round((r1 - x1).astype(np.float32))
    return x0, x1, x2


def emulate_split_gemm(a, b, terms=3):
    """FP64 value of the kept term products of an (M,K) x (K,N) product.

    terms=1: plain BF16 operands; terms=2: the 3-product scheme; terms=3: six products.
    Accumulation is exact (FP64), so this isolates the operand-splitting error.
    """
    sa = split3(a)[:terms]
    sb = split3(b)[:terms]
    out = np.zeros((a.shape[0], b.shape[1]))
    for i in range(terms):
        for j in range(terms):
            if i + j < terms:
                out += sa[i].astype(np.float64) @ sb[j].astype(np.float64)
    return out
