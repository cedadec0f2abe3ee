"""Pins of the oracle's BF16 rounding model and the 3-term split."""
import numpy as np
import torch

import oracle


def test_bf16_round_matches_torch_conversion():
    rng = np.random.default_rng(1)
    x = (rng.standard_normal(1 << 16) * np.exp(rng.uniform(-20, 20, 1 << 16))).astype(np.float32)
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float32).numpy()
    np.testing.assert_array_equal(oracle.bf16_round(x), ref)


def test_bf16_round_ties_to_even():
    one = np.float32(1.0)
    ulp = np.float32(2.0 ** -7)
    assert oracle.bf16_round(np.float32(one + ulp / 2)) == one              # tie -> even (1.0)
    assert oracle.bf16_round(np.float32(one + 3 * ulp / 2)) == one + 2 * ulp  # tie -> even (up)


def test_three_term_split_is_exact_for_normal_fp32():
    rng = np.random.default_rng(2)
    x = rng.standard_normal(1 << 18).astype(np.float32)
    x0, x1, x2 = oracle.split3(x)
    back = x0.astype(np.float64) + x1.astype(np.float64) + x2.astype(np.float64)
    np.testing.assert_array_equal(back, x.astype(np.float64))
    for t in (x0, x1, x2):
        np.testing.assert_array_equal(oracle.bf16_round(t), t)


def test_split_product_error_ordering():
    rng = np.random.default_rng(3)
    a = rng.standard_normal((64, 256)).astype(np.float32)
    b = rng.standard_normal((256, 48)).astype(np.float32)
    ref = a.astype(np.float64) @ b.astype(np.float64)
    errs = [np.linalg.norm(oracle.emulate_split_gemm(a, b, t) - ref) / np.linalg.norm(ref) for t in (1, 2, 3)]
    assert errs[0] > 1e-3 and 1e-7 < errs[1] < 1e-4 and errs[2] < 1e-7
