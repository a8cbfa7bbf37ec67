"""Pins of the oracle side's 16-bit storage rounding (tests/gpu_util.round_storage).

The 16-bit payload forms store every leaf coefficient rounded to nearest even
from float32; the oracle renders the rounded values to isolate the arithmetic.
These tests hold that rounding against conversions written elsewhere: torch's
float32 -> bfloat16 and float32 -> float16 casts (IEEE round-to-nearest-even),
on special values and on random bit patterns that include exact ties."""
import numpy as np
import pytest
import torch

from paper_2202_06088_amd import _lib
from gpu_util import round_storage


def _special_f32():
    f = np.float32
    tiny = np.finfo(np.float32).tiny
    vals = [0.0, -0.0, np.inf, -np.inf, np.nan, 1.0, -1.0, np.finfo(np.float32).max, -np.finfo(np.float32).max,
            tiny, -tiny, tiny / 2, tiny * (1 - 2.0 ** -23), 2.0 ** -149, -2.0 ** -149,
            # bfloat16 ties: exactly half way between two bfloat16 values, both parities
            1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8, -(1.0 + 2.0 ** -8), 2.0 ** -130 * (1 + 2.0 ** -8),
            # float16 ties, subnormals and overflow
            1.0 + 2.0 ** -11, 1.0 + 3 * 2.0 ** -11, 2.0 ** -24, 2.0 ** -25, 3 * 2.0 ** -25, 65504.0, 65519.0,
            65520.0, -65520.0, 1e5]
    out = np.array(vals, np.float64).astype(f)
    # the largest float32 values round past the largest finite bfloat16: +-inf
    big = np.array([0x7F7F8000, 0x7F7FFFFF, 0xFF7F8000, 0x7F7F7FFF], np.uint32).view(np.float32)
    return np.concatenate([out, big])


def _random_f32(n, seed):
    rng = np.random.default_rng(seed)
    bits = rng.integers(0, 2 ** 32, n, dtype=np.uint64).astype(np.uint32)
    # a quarter of them exact bfloat16 ties (low half = 0x8000)
    bits[: n // 4] = (bits[: n // 4] & 0xFFFF0000) | 0x8000
    return bits.view(np.float32)


def _same(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    nan = np.isnan(b)
    assert np.array_equal(np.isnan(a), nan)
    # bit equality of the finite and infinite values, signed zeros included
    assert np.array_equal(a[~nan].view(np.uint64), b[~nan].view(np.uint64))


@pytest.mark.parametrize("src", ["special", "random"])
def test_bf16_rounding_matches_torch(src):
    x = _special_f32() if src == "special" else _random_f32(2_000_000, 5)
    ref = torch.from_numpy(x.copy()).to(torch.bfloat16).to(torch.float64).numpy()
    _same(round_storage(x, _lib.BF16), ref)


@pytest.mark.parametrize("src", ["special", "random"])
def test_f16_rounding_matches_torch(src):
    x = _special_f32() if src == "special" else _random_f32(2_000_000, 6)
    ref = torch.from_numpy(x.copy()).to(torch.float16).to(torch.float64).numpy()
    _same(round_storage(x, _lib.F16), ref)


def test_rounding_spot_values():
    # values fixed by the formats themselves
    x = np.array([1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8, 1.0 + 2.0 ** -11, 65520.0, 2.0 ** -25], np.float32)
    assert round_storage(x[:2], _lib.BF16).tolist() == [1.0, 1.0 + 2.0 ** -6]
    assert round_storage(x[2:], _lib.F16).tolist() == [1.0, np.inf, 0.0]
    assert np.array_equal(round_storage(x, _lib.F32), x.astype(np.float64))
