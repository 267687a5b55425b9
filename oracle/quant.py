"""Reduced-precision staging of the data (test infrastructure only).

The low-precision forms of the method store the tall data in BF16, or in
FP8 E4M3 with one power-of-two scale per column, before the sketch and the
data products read it.  These are plain definitions of those encodings:

* BF16: the float32 values with zero low 16 bits; encoding picks the
  nearer of the two neighbouring BF16 values by exact comparison, ties to
  the even significand, overflowing to infinity as IEEE round-to-nearest
  does; a NaN keeps its sign and upper payload with the quiet bit set.
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

Parity status: pinned.  Tests check hand-worked ties, the unit roundoff
bounds, subnormals, saturation, the largest values, NaN and infinities,
and (BF16) an exhaustive sweep of neighbouring float32 patterns against a
brute-force search over the ordered BF16 values.
"""
from __future__ import annotations

import numpy as np

FP8_MAX = 448.0


def bf16_round(x) -> np.ndarray:
    """float32 -> nearest BF16 value (ties to the even significand), returned
    as float32, by exact comparison with the two neighbouring BF16 values.

    BF16 values are the float32 values whose low 16 bits are zero.  For a
    finite x the neighbours are lo (x with its low 16 bits cleared: the next
    BF16 value towards zero) and hi (the next BF16 value away from zero).
    Both distances are computed exactly in float64; the nearer one wins, a
    tie goes to the neighbour whose last significand bit is 0.  Past the
    largest finite BF16 value (2 - 2^-7) 2^127 the upper neighbour is
    infinity, taken at 2^128 for the comparison (IEEE overflow of
    round-to-nearest).  +-0 and +-inf are kept.  A NaN stays a NaN: its upper
    16 bits with the quiet bit (bit 6 of the BF16 significand) set, so the
    sign and the high payload bits are kept."""
    x32 = np.ascontiguousarray(x, dtype=np.float32)
    u = x32.view(np.uint32).astype(np.uint64)
    sign = u & np.uint64(0x80000000)
    mag = u & np.uint64(0x7FFFFFFF)
    out = np.empty_like(u)
    nan = mag > np.uint64(0x7F800000)
    out[nan] = ((u[nan] >> np.uint64(16)) | np.uint64(0x40)) << np.uint64(16)
    fin = ~nan
    lo_bits = mag[fin] & np.uint64(0xFFFF0000)
    hi_bits = lo_bits + np.uint64(0x10000)
    v = np.abs(x32[fin].astype(np.float64))
    lo = lo_bits.astype(np.uint32).view(np.float32).astype(np.float64)
    hi = np.where(hi_bits >= np.uint64(0x7F800000), 2.0 ** 128,
                  np.minimum(hi_bits, np.uint64(0x7F7FFFFF)).astype(np.uint32).view(np.float32).astype(np.float64))
    with np.errstate(invalid="ignore"):
        dlo = v - lo
        dhi = hi - v
    even_hi = ((hi_bits >> np.uint64(16)) & np.uint64(1)) == 0
    pick_hi = np.isfinite(v) & ((dhi < dlo) | ((dhi == dlo) & even_hi))
    res = np.where(pick_hi, np.minimum(hi_bits, np.uint64(0x7F800000)), lo_bits)
    out[fin] = res | sign[fin]
    return out.astype(np.uint32).view(np.float32)


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
