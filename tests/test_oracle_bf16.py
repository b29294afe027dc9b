"""Pins for the bf16 emulation used by reduced-precision sketch tests:
round-to-nearest-even against torch's float32 -> bfloat16 conversion (an
independent library routine), and the split x = hi + lo being exact."""
import numpy as np
import torch

from oracle.bf16 import matmul_bf16x3, split3, to_bf16


def test_to_bf16_matches_torch_rne():
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.standard_normal(200000).astype(np.float32) * 10.0 ** rng.integers(-20, 20, 200000),
                        np.array([0.0, -0.0, 1.0, 1.00390625, 1.01171875, 3.0e38, -1e-40], np.float32)])
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float32).numpy()
    np.testing.assert_array_equal(to_bf16(x), ref)


def test_split3_is_exact_and_small():
    x = np.random.default_rng(1).standard_normal(100000).astype(np.float32)
    hi, lo = split3(x)
    np.testing.assert_array_equal(to_bf16(hi), hi)
    np.testing.assert_array_equal(to_bf16(lo), lo)
    assert np.all(np.abs(lo) <= np.abs(hi) * 2.0 ** -8)
    # the dropped lo*lo term bounds the error of the 3-term product
    A = np.random.default_rng(2).standard_normal((64, 200)).astype(np.float32)
    B = np.random.default_rng(3).standard_normal((200, 16)).astype(np.float32)
    exact = A.astype(np.float64) @ B.astype(np.float64)
    assert np.max(np.abs(matmul_bf16x3(A, B) - exact)) <= 200 * 2.0 ** -16 * 16
