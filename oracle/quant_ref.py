"""Reference encodings of the reduced-precision sweeps -- TEST INFRASTRUCTURE, NOT PRODUCT CODE.

Plain numpy versions of the three storage formats, written from their published definitions
and kept deliberately naive so that they can be read against those definitions:

* bfloat16: the upper 16 bits of an IEEE binary32 value (1 sign, 8 exponent, 7 fraction bits),
  rounded to nearest with ties to even.
* binary16 (FP16): IEEE 754 half precision, round to nearest even; numpy's float16 cast is the
  library routine for it.
* FP8 E4M3 as defined in the OCP 8-bit floating point specification (v1.0): 1 sign, 4 exponent
  (bias 7), 3 mantissa bits; exponent field 0 holds subnormals m * 2^-9; the all-ones pattern
  S.1111.111 is NaN; there are no infinities; the largest finite magnitude is 448.  Conversion
  rounds to nearest (ties to the even code) and saturates at +-448, and the values are divided
  by a per-slice FP32 scale amax / 448 first (the scaling recipe of the sweep's FP8 variant).

The encoder for E4M3 searches the table of all representable values (brute force), so it
shares nothing with the bit-manipulation encoder of the HIP library.
"""

from __future__ import annotations

import numpy as np

E4M3_MAX = 448.0


def bf16_round(x):
    """Round float32 values to the nearest bfloat16 (ties to even); returned as float32."""
    x = np.ascontiguousarray(x, dtype=np.float32)
    u = x.view(np.uint32).astype(np.uint64)
    nan = np.isnan(x)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) & 0xFFFF0000).astype(np.uint32)
    out = r.view(np.float32).copy()
    out[nan] = np.nan
    return out


def f16_round(x):
    """Round float32 values to IEEE binary16 (numpy's cast rounds to nearest even)."""
    return np.asarray(x, dtype=np.float32).astype(np.float16).astype(np.float32)


def e4m3_decode_table():
    """Value of every one of the 256 E4M3 codes (NaN for the two NaN codes)."""
    vals = np.empty(256, dtype=np.float64)
    for code in range(256):
        sign = -1.0 if code & 0x80 else 1.0
        e = (code >> 3) & 0xF
        m = code & 0x7
        if e == 0xF and m == 0x7:
            vals[code] = np.nan
        elif e == 0:
            vals[code] = sign * m * 2.0 ** -9
        else:
            vals[code] = sign * (1.0 + m / 8.0) * 2.0 ** (e - 7)
    return vals


_TABLE = e4m3_decode_table()
# non-negative finite codes 0x00..0x7E in increasing value
_POS_CODES = np.arange(0x7F)
_POS_VALS = _TABLE[_POS_CODES]


def e4m3_encode(x):
    """Nearest E4M3 code (ties to the even code, saturating at 448) of each float value."""
    x = np.asarray(x, dtype=np.float64)
    out = np.empty(x.shape, dtype=np.uint8)
    flat_x = x.ravel()
    flat_o = out.ravel()
    for i, v in enumerate(flat_x):
        if np.isnan(v):
            flat_o[i] = 0x7F
            continue
        sign = 0x80 if np.signbit(v) else 0
        a = min(abs(v), E4M3_MAX)
        j = int(np.searchsorted(_POS_VALS, a))     # first value >= a
        if j < len(_POS_VALS) and _POS_VALS[j] == a:
            code = int(_POS_CODES[j])
        else:
            lo, hi = j - 1, j
            dlo, dhi = a - _POS_VALS[lo], _POS_VALS[hi] - a
            if dlo < dhi:
                code = int(_POS_CODES[lo])
            elif dhi < dlo:
                code = int(_POS_CODES[hi])
            else:
                code = int(_POS_CODES[lo] if _POS_CODES[lo] % 2 == 0 else _POS_CODES[hi])
        flat_o[i] = sign | code
    return out


def e4m3_decode(codes):
    return _TABLE[np.asarray(codes, dtype=np.uint8)]


def fp8_slice_scales(x2d):
    """Per-column scale amax / 448 of a (rows, L) float32 matrix, in float32 (1 for a zero column)."""
    x2d = np.asarray(x2d, dtype=np.float32)
    amax = np.max(np.abs(x2d), axis=0).astype(np.float32)
    s = (amax / np.float32(E4M3_MAX)).astype(np.float32)
    s[amax == 0] = np.float32(1.0)
    return s


def fp8_round_scaled(x2d, scales):
    """dec(enc(x / s)) * s per column, every step in float32 as the storage path does."""
    x2d = np.asarray(x2d, dtype=np.float32)
    q = (x2d / scales[None, :]).astype(np.float32)
    d = e4m3_decode(e4m3_encode(q)).astype(np.float32)
    return (d * scales[None, :]).astype(np.float32)


def quantize(x2d, precision):
    """The storage round trip of a (rows, L) float32 matrix: (values, scales or None)."""
    if precision == "bf16":
        return bf16_round(x2d), None
    if precision == "fp16":
        return f16_round(x2d), None
    if precision == "fp8":
        s = fp8_slice_scales(x2d)
        return fp8_round_scaled(x2d, s), s
    raise ValueError(precision)
