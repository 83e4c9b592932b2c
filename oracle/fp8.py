"""FP8 storage of the coupling matrix, written from the format definitions --
TEST INFRASTRUCTURE (see oracle/__init__.py for the rules).

OCP 8-bit floating point, E4M3 (e4m3fn): 1 sign bit, 4 exponent bits with
bias 7, 3 mantissa bits.  Exponent field 0 holds the subnormals m * 2^-9;
exponent field 1..15 holds (1 + m/8) * 2^(E-7), except that 0x7f and 0xff
(all exponent and mantissa bits set) are NaN; there are no infinities, so
the largest finite value is 0x7e = 448.  OCP E8M0 (the shared-scale format
of the microscaling specification): one byte E, value 2^(E-127), 0xff NaN.

Row quantization of J (the library's CHYM_J_FP8): per row p, e_p = the least
integer with max_q |J_pq| <= 448 * 2^e_p (0 for an all-zero row); q_pq =
J_pq / 2^e_p rounded to the nearest E4M3 value, ties to the even code (the
one with mantissa bit 0).  A row with a non-finite value or with e_p outside
[-127, 127] gets E = 0xff and codes 0x7f.

Encoding here searches the sorted table of E4M3 values (nearest neighbour,
ties to even code); pinned in tests/test_oracle_fp8.py by the format's fixed
values and by a library conversion.
"""
from __future__ import annotations

import math

import numpy as np


def e4m3_table() -> np.ndarray:
    """float64 value of every code 0..255."""
    out = np.empty(256, dtype=np.float64)
    for code in range(256):
        sign = -1.0 if code & 0x80 else 1.0
        e = (code >> 3) & 0xF
        m = code & 0x7
        if (code & 0x7F) == 0x7F:
            out[code] = math.nan
        elif e == 0:
            out[code] = sign * m * 2.0 ** -9
        else:
            out[code] = sign * (1.0 + m / 8.0) * 2.0 ** (e - 7)
    return out


_TABLE = e4m3_table()
_POS = _TABLE[:0x7F]  # codes 0x00 .. 0x7e: 0, subnormals, normals up to 448, increasing


def e4m3_encode(v) -> np.ndarray:
    """Nearest E4M3 code of each value (|v| <= 448), ties to the even code;
    the sign bit follows the value's sign bit (so -0.0 -> 0x80)."""
    v = np.asarray(v, dtype=np.float64)
    a = np.abs(v)
    if np.any(a > 448.0) or np.any(~np.isfinite(a)):
        raise ValueError("e4m3_encode needs finite |v| <= 448")
    hi = np.searchsorted(_POS, a, side="left")  # first table value >= a
    hi = np.minimum(hi, len(_POS) - 1)
    lo = np.maximum(hi - 1, 0)
    d_lo = a - _POS[lo]
    d_hi = _POS[hi] - a
    pick_hi = (d_hi < d_lo) | ((d_hi == d_lo) & (hi % 2 == 0))
    code = np.where(pick_hi, hi, lo)
    code = np.where(a == _POS[hi], hi, code)  # exact hits (also a == 0)
    neg = np.signbit(v)
    return (code | np.where(neg, 0x80, 0)).astype(np.uint8)


def row_exponent(amax: float) -> int:
    """Least integer e with amax <= 448 * 2^e (0 for amax == 0)."""
    if amax == 0.0:
        return 0
    e = math.ceil(math.log2(amax / 448.0))
    # guard the floating log: step to the exact least e
    while amax > 448.0 * 2.0 ** e:
        e += 1
    while amax <= 448.0 * 2.0 ** (e - 1):
        e -= 1
    return e


def quantize(J):
    """float32 J [n][n] -> (codes uint8 [n][n], E8M0 exponents uint8 [n])."""
    J = np.asarray(J, dtype=np.float32)
    n = J.shape[0]
    codes = np.empty((n, n), dtype=np.uint8)
    expo = np.empty(n, dtype=np.uint8)
    for p in range(n):
        row = J[p].astype(np.float64)
        if not np.all(np.isfinite(row)):
            codes[p] = 0x7F
            expo[p] = 0xFF
            continue
        e = row_exponent(float(np.max(np.abs(row))))
        if e < -127 or e > 127:
            codes[p] = 0x7F
            expo[p] = 0xFF
            continue
        codes[p] = e4m3_encode(row * 2.0 ** (-e))
        expo[p] = e + 127
    return codes, expo


def decode(codes, expo) -> np.ndarray:
    """Couplings J_pq = e4m3(codes[p, q]) * 2^(E_p - 127) as float64."""
    codes = np.asarray(codes, dtype=np.uint8)
    expo = np.asarray(expo, dtype=np.uint8)
    scale = np.where(expo == 0xFF, math.nan, np.ldexp(1.0, expo.astype(np.int64) - 127))
    return _TABLE[codes] * scale[:, None]


def pack(codes, expo) -> np.ndarray:
    """The library's byte layout: [n + 1][n], codes then the exponent row."""
    return np.concatenate([np.asarray(codes, np.uint8), np.asarray(expo, np.uint8)[None, :]], axis=0)
