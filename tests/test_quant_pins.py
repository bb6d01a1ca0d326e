"""Pins of the reference encodings (oracle/quant_ref.py) against the format definitions.

bfloat16 and binary16 are checked on hand-derived rounding cases and against numpy's IEEE
half cast; E4M3 against the values the OCP FP8 specification fixes (largest finite 448,
smallest subnormal 2^-9, smallest normal 2^-6, the NaN pattern) and by exhaustive round trips.
"""

import numpy as np
import pytest

from oracle import quant_ref as q


def test_bf16_hand_cases():
    cases = {
        1.0 + 2.0 ** -8: 1.0,                      # midpoint of 1 and 1 + 2^-7: tie to the even mantissa (1)
        1.0 + 3 * 2.0 ** -8: 1.0 + 2.0 ** -6,      # midpoint of 1+2^-7 (odd) and 1+2^-6 (even)
        1.0 + 2.0 ** -8 + 2.0 ** -20: 1.0 + 2.0 ** -7,   # just above the midpoint
        -2.5: -2.5,
        0.0: 0.0,
    }
    for x, want in cases.items():
        got = float(q.bf16_round(np.array([x], dtype=np.float32))[0])
        assert got == want, (x, got, want)
    assert np.isnan(q.bf16_round(np.array([np.nan], dtype=np.float32))[0])


def test_bf16_properties():
    rng = np.random.default_rng(0)
    x = (rng.standard_normal(20000) * np.exp(rng.uniform(-20, 20, 20000))).astype(np.float32)
    r = q.bf16_round(x)
    assert np.all((r.view(np.uint32) & 0xFFFF) == 0)            # a bfloat16 value
    ulp = np.ldexp(np.float64(1.0), np.frexp(np.abs(x).astype(np.float64))[1] - 8)
    assert np.all(np.abs(r.astype(np.float64) - x) <= ulp / 2 + 1e-300)


def test_f16_is_ieee_half():
    assert q.f16_round(np.array([65504.0, 1.0 + 2.0 ** -11, 2.0 ** -24], dtype=np.float32)).tolist() == \
        [65504.0, 1.0, 2.0 ** -24]


def test_e4m3_table_matches_the_spec():
    t = q.e4m3_decode_table()
    assert t[0x7E] == 448.0 and t[0xFE] == -448.0
    assert t[0x01] == 2.0 ** -9 and t[0x08] == 2.0 ** -6 and t[0x07] == 7 * 2.0 ** -9
    assert t[0x38] == 1.0 and t[0x3F] == 1.875 and t[0x40] == 2.0
    assert np.isnan(t[0x7F]) and np.isnan(t[0xFF])
    assert np.sum(np.isnan(t)) == 2
    pos = t[:0x7F]
    assert np.all(np.diff(pos) > 0)                              # codes are ordered by value


def test_e4m3_round_trip_and_rounding():
    t = q.e4m3_decode_table()
    codes = np.array([c for c in range(256) if not np.isnan(t[c]) and c != 0x80], dtype=np.uint8)
    assert np.array_equal(q.e4m3_encode(t[codes]), codes)
    # ties go to the even code; above 448 saturates; small values go to subnormals / zero
    assert q.e4m3_decode(q.e4m3_encode([15.5, 17.0, 460.0, 1e6, -1e6, 2.0 ** -10, 3 * 2.0 ** -10, 1e-9])).tolist() \
        == [16.0, 16.0, 448.0, 448.0, -448.0, 0.0, 2 * 2.0 ** -9, 0.0]


def test_e4m3_nearest_on_random_values():
    rng = np.random.default_rng(1)
    x = rng.uniform(-500, 500, 5000)
    got = q.e4m3_decode(q.e4m3_encode(x))
    t = q.e4m3_decode_table()
    finite = t[~np.isnan(t)]
    best = np.min(np.abs(np.clip(x, -448, 448)[:, None] - finite[None, :]), axis=1)
    assert np.allclose(np.abs(np.clip(x, -448, 448) - got), best, rtol=0, atol=0)


@pytest.mark.parametrize("prec", ["bf16", "fp16", "fp8"])
def test_quantize_relative_error(prec):
    rng = np.random.default_rng(2)
    x = rng.uniform(-1, 1, (300, 7)).astype(np.float32) * np.array([1, 10, 1e-3, 5, 0.5, 2, 100], np.float32)
    r, s = q.quantize(x, prec)
    bound = {"bf16": 2.0 ** -8, "fp16": 2.0 ** -11, "fp8": 2.0 ** -4}[prec]
    big = np.abs(x) > (np.max(np.abs(x), axis=0) * 2.0 ** -6 if prec == "fp8" else 1e-4)
    assert np.all(np.abs(r[big] - x[big]) <= bound * np.abs(x[big]) * (1 + 1e-6))
    if prec == "fp8":
        assert np.allclose(s, np.max(np.abs(x), axis=0) / 448.0, rtol=1e-7)
        assert np.all(np.abs(r) <= 448.0 * s[None, :] * (1 + 1e-6))
