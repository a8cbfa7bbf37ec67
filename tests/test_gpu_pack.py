"""Bit-exact check of the storage conversion on the GPU (neuvv_pack_leaves,
neuvv_pack_rows): FP32 -> FP16 / BF16 with round-to-nearest-even, placed in
the payload layout the header documents, padding zero.

The expected bytes are built on the host from torch's CPU casts (IEEE
round-to-nearest-even, independent of the library's conversion) and the
header's element formulas:
  leaf rows:   value r of slot s at element s * NG * V + r
  vector SoA:  value r of slot s at element (r / V) * N * V + s * V + r % V
with V = 4 (FP32) or 8 (16-bit) values per 16-byte vector and NG = ceil(R / V).
The inputs hold seeded N(0, s) coefficients with special values planted:
signed zeros, subnormals of both formats, exact ties, the largest finite
values, values that round past them to infinity, infinities and NaN (NaN is
compared as NaN, its payload bits being free)."""
import numpy as np
import pytest
import torch

from gpu_util import DEV, announce
from paper_2202_06088_amd import _lib

pytestmark = pytest.mark.gpu

_BITS = {_lib.F32: (torch.float32, torch.int32, np.uint32), _lib.F16: (torch.float16, torch.int16, np.uint16),
         _lib.BF16: (torch.bfloat16, torch.int16, np.uint16)}
_NAMES = {_lib.F32: "f32", _lib.F16: "f16", _lib.BF16: "bf16"}


def _specials():
    big_bf = np.array([0x7F7F8000, 0x7F7FFFFF, 0xFF7F8000, 0x7F7F7FFF], np.uint32).view(np.float32)
    vals = [0.0, -0.0, np.inf, -np.inf, np.nan, 2.0 ** -149, -2.0 ** -149, np.finfo(np.float32).tiny,
            1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8, 1.0 + 2.0 ** -11, 1.0 + 3 * 2.0 ** -11, 2.0 ** -24, 2.0 ** -25,
            3 * 2.0 ** -25, 65504.0, 65519.0, 65520.0, -65520.0, 1e5, np.finfo(np.float32).max]
    return np.concatenate([np.array(vals, np.float64).astype(np.float32), big_bf])


def _values(rng, n, R, s):
    a = rng.normal(0.0, s, (n, R)).astype(np.float32)
    sp = _specials()
    flat = a.reshape(-1)
    where = rng.choice(flat.size, size=min(flat.size, 8 * sp.size), replace=False)
    flat[where] = np.resize(sp, where.size)
    # random bfloat16 and float16 ties
    t = rng.choice(flat.size, size=flat.size // 16, replace=False)
    bits = flat[t].view(np.uint32)
    half = t.size // 2
    flat[t[:half]] = ((bits[:half] & 0xFFFF0000) | 0x8000).view(np.float32)
    # float16 ties: the midpoint of two neighbouring finite float16 values (exact in float32)
    h = rng.integers(0, 0x7BFF, t.size - half).astype(np.uint16)
    lo = h.view(np.float16).astype(np.float32)
    hi = (h + 1).astype(np.uint16).view(np.float16).astype(np.float32)
    sign = np.where(rng.random(h.size) < 0.5, -1.0, 1.0).astype(np.float32)
    flat[t[half:]] = sign * (lo + (hi - lo) * np.float32(0.5))
    return a


def _host_round_bits(x: np.ndarray, dtype: int) -> np.ndarray:
    td, ti, nt = _BITS[dtype]
    return torch.from_numpy(np.ascontiguousarray(x, np.float32)).to(td).view(ti).numpy().view(nt)


def _expected(x: np.ndarray, slots: np.ndarray, dtype: int, layout: int) -> np.ndarray:
    """Elements of the packed array: rounded value r of input leaf i at slot slots[i]."""
    n, R = x.shape
    V = 4 if dtype == _lib.F32 else 8
    NG = -(-R // V)
    nt = _BITS[dtype][2]
    out = np.zeros(NG * n * V, nt)
    rb = _host_round_bits(x, dtype)
    r = np.arange(R)
    for i in range(n):
        s = int(slots[i])
        if layout == _lib.LAYOUT_LEAF_ROWS:
            idx = s * NG * V + r
        else:
            idx = (r // V) * n * V + s * V + r % V
        out[idx] = rb[i]
    return out


def _compare(got_t: torch.Tensor, want: np.ndarray, dtype: int, label: str):
    td, ti, nt = _BITS[dtype]
    got = got_t.view(ti).cpu().numpy().view(nt)
    assert got.shape == want.shape, (got.shape, want.shape)
    f = np.float32 if dtype == _lib.F32 else np.float16
    if dtype == _lib.BF16:
        gnan = np.isnan((got.astype(np.uint32) << 16).view(np.float32))
        wnan = np.isnan((want.astype(np.uint32) << 16).view(np.float32))
    else:
        gnan = np.isnan(got.view(f))
        wnan = np.isnan(want.view(f))
    assert np.array_equal(gnan, wnan), label
    diff = int((got[~wnan] != want[~wnan]).sum())
    announce(f"{label}: {got.size} elements, {int(wnan.sum())} NaN, {diff} differing")
    assert diff == 0, label


@pytest.mark.parametrize("dtype", [_lib.F32, _lib.F16, _lib.BF16])
@pytest.mark.parametrize("layout", [_lib.LAYOUT_LEAF_ROWS, _lib.LAYOUT_VEC_SOA])
@pytest.mark.parametrize("K,C", [(16, 8), (14, 31), (30, 8)])
def test_pack_leaves_bit_exact(dtype, layout, K, C):
    rng = np.random.default_rng(100 + 7 * dtype + layout + K)
    n = 1237   # not a multiple of any vector or block size
    hh = _values(rng, n, 3 * K, 0.3)
    ws = _values(rng, n, C, 1.0)
    slots = rng.permutation(n).astype(np.int64)
    a, b = _lib.neuvv_payload_words(K, C, dtype, n)
    td = _BITS[dtype][0]
    hh_out = torch.full((a,), 7.0, dtype=td, device=DEV)    # padding must be written with zero
    ws_out = torch.full((b,), 7.0, dtype=td, device=DEV)
    _lib.neuvv_pack_leaves(K, C, dtype, layout, n, torch.from_numpy(hh).to(DEV), torch.from_numpy(ws).to(DEV),
                           torch.from_numpy(slots).to(DEV), hh_out, ws_out)
    torch.cuda.synchronize()
    tag = f"pack K={K} C={C} {_NAMES[dtype]} layout={layout}"
    _compare(hh_out, _expected(hh, slots, dtype, layout), dtype, tag + " hh")
    _compare(ws_out, _expected(ws, slots, dtype, layout), dtype, tag + " wsig")


@pytest.mark.parametrize("dtype", [_lib.F32, _lib.F16, _lib.BF16])
@pytest.mark.parametrize("layout", [_lib.LAYOUT_LEAF_ROWS, _lib.LAYOUT_VEC_SOA])
@pytest.mark.parametrize("R", [1, 9, 31])
def test_pack_rows_bit_exact(dtype, layout, R):
    rng = np.random.default_rng(300 + 7 * dtype + layout + R)
    n = 515
    x = _values(rng, n, R, 2.0)
    V = 4 if dtype == _lib.F32 else 8
    out = torch.full((-(-R // V) * n * V,), 7.0, dtype=_BITS[dtype][0], device=DEV)
    # identity slot order (slot_of_input NULL)
    _lib.neuvv_pack_rows(R, dtype, layout, n, torch.from_numpy(x).to(DEV), None, out)
    torch.cuda.synchronize()
    _compare(out, _expected(x, np.arange(n), dtype, layout), dtype,
             f"pack_rows R={R} {_NAMES[dtype]} layout={layout}")
