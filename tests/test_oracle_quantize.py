"""Pins for oracle.quantize: bfloat16 round-to-nearest-even against known
bit patterns and against torch's CPU float32 -> bfloat16 conversion."""
import numpy as np
import torch

from oracle import quantize as q


def test_known_values():
    x = np.array([1.0, -2.0, 0.0, 3.140625, 1.00390625, 1.01171875, 65504.0, np.inf], dtype=np.float32)
    b = q.to_bf16_bits(x)
    # 1.00390625 = 1 + 2^-8 is a tie between 1 and 1 + 2^-7: rounds to even (1.0)
    # 1.01171875 = 1 + 3 * 2^-8 is a tie between 1 + 2^-7 and 1 + 2^-6: rounds to even (1 + 2^-6)
    np.testing.assert_array_equal(
        q.bf16_bits_to_f64(b), [1.0, -2.0, 0.0, 3.140625, 1.0, 1.015625, 65536.0, np.inf])
    assert np.isnan(q.round_to_bf16(np.array([np.nan], dtype=np.float32)))[0]


def test_matches_torch_rne():
    rng = np.random.default_rng(0)
    x = (rng.standard_normal(200000) * 10.0 ** rng.integers(-30, 30, 200000)).astype(np.float32)
    ours = q.to_bf16_bits(x)
    ref = torch.from_numpy(x).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    np.testing.assert_array_equal(ours, ref)


def test_relative_error_bound():
    rng = np.random.default_rng(1)
    x = rng.standard_normal(100000).astype(np.float32)
    y = q.round_to_bf16(x)
    assert np.all(np.abs(y - x) <= 2.0 ** -8 * np.abs(x))
