"""Reduced-precision staging of the data (test infrastructure only).

The low-precision forms of the method store the tall data in BF16, or in
FP8 E4M3 with one power-of-two scale per column, before the sketch and the
data products read it.  These are plain definitions of those encodings:

* BF16: the upper 16 bits of an IEEE binary32 value after rounding to
  nearest, ties to even, on the discarded 16 bits.
* FP8 E4M3 (the OCP 8-bit format with 4 exponent bits, bias 7, 3 mantissa
  bits, no infinities, the all-ones pattern is NaN): the finite values are
  (-1)^s (m/8) 2^-6 for e = 0 and (-1)^s (1 + m/8) 2^(e-7) for e = 1..15
  except (e, m) = (15, 7); the largest is 448.  Encoding rounds to the
  nearest finite value, ties to the even mantissa, and saturates at +-448.
* Column scale: 2^ceil(log2(max_i |x_ij| / 448)) (1 for an all-zero
  column), so every scaled entry lies within the FP8 range and undoing the
  scale is exact.

The FP8 rounding is done by brute force over the table of all finite
values, so it can be read against the definition directly.
"""
from __future__ import annotations

import numpy as np

FP8_MAX = 448.0


def bf16_round(x) -> np.ndarray:
    """float32 -> nearest BF16 (ties to even), returned as float32."""
    u = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    bias = 0x7FFF + ((u >> 16) & 1)
    r = ((u + bias) >> 16) << 16
    return r.astype(np.uint32).view(np.float32)


def fp8_e4m3_table():
    """All finite non-negative E4M3 values with their codes (ascending)."""
    vals, codes = [], []
    for e in range(16):
        for m in range(8):
            if e == 15 and m == 7:
                continue   # NaN pattern
            v = (m / 8.0) * 2.0 ** -6 if e == 0 else (1.0 + m / 8.0) * 2.0 ** (e - 7)
            vals.append(v)
            codes.append((e << 3) | m)
    order = np.argsort(vals, kind="stable")
    return np.array(vals)[order], np.array(codes, dtype=np.uint8)[order]


_FP8_VALS, _FP8_CODES = fp8_e4m3_table()


def fp8_e4m3_encode(x) -> np.ndarray:
    """Round to the nearest E4M3 value (ties to even mantissa), saturating at
    +-448; returns the 8-bit codes."""
    x = np.asarray(x, dtype=np.float64)
    a = np.minimum(np.abs(x), FP8_MAX)
    hi = np.searchsorted(_FP8_VALS, a, side="left")            # first value >= a
    hi = np.minimum(hi, len(_FP8_VALS) - 1)
    lo = np.maximum(hi - 1, 0)
    dlo, dhi = a - _FP8_VALS[lo], _FP8_VALS[hi] - a
    pick_hi = (dhi < dlo) | ((dhi == dlo) & ((_FP8_CODES[hi] & 1) == 0) & (hi != lo))
    idx = np.where(pick_hi, hi, lo)
    idx = np.where(_FP8_VALS[hi] == a, hi, idx)
    code = _FP8_CODES[idx]
    sign = (np.signbit(x) & (_FP8_VALS[idx] != 0.0)).astype(np.uint8) << 7
    return (code | sign).astype(np.uint8)


def fp8_e4m3_decode(code) -> np.ndarray:
    c = np.asarray(code, dtype=np.uint8).astype(np.int64)
    s = np.where(c & 0x80, -1.0, 1.0)
    e = (c >> 3) & 0xF
    m = c & 7
    v = np.where(e == 0, (m / 8.0) * 2.0 ** -6, (1.0 + m / 8.0) * np.exp2(e - 7.0))
    v = np.where((e == 15) & (m == 7), np.nan, v)
    return s * v


def fp8_column_scales(X) -> np.ndarray:
    """Per-column power-of-two scales (float64): the smallest 2^e with
    max |x| <= 448 2^e, found by exact comparisons."""
    amax = np.max(np.abs(np.asarray(X, dtype=np.float64)), axis=0)
    out = np.ones_like(amax)
    for j, a in enumerate(amax):
        if a > 0:
            e = int(np.ceil(np.log2(a / FP8_MAX)))
            while a > FP8_MAX * 2.0 ** e:
                e += 1
            while a <= FP8_MAX * 2.0 ** (e - 1):
                e -= 1
            out[j] = 2.0 ** e
    return out


def fp8_stage(X):
    """(codes n x d uint8, scales d float64) with X ~ decode(codes) * scales."""
    sc = fp8_column_scales(X)
    return fp8_e4m3_encode(np.asarray(X, dtype=np.float64) / sc[None, :]), sc


def fp8_unstage(codes, scales) -> np.ndarray:
    return fp8_e4m3_decode(codes) * np.asarray(scales)[None, :]
