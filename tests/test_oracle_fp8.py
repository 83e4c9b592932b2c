"""Pins of the oracle's FP8 coupling storage: the E4M3 format's fixed values,
PyTorch's own float8_e4m3fn conversion (an independent implementation of the
same OCP format), round-to-nearest-even ties, and the row-exponent rule."""
import math

import numpy as np
import pytest

from oracle import fp8

torch = pytest.importorskip("torch")


def test_fixed_values_of_the_format():
    t = fp8.e4m3_table()
    assert t[0x7E] == 448.0                      # largest finite
    assert t[0x08] == 2.0 ** -6                  # smallest normal
    assert t[0x01] == 2.0 ** -9                  # smallest subnormal
    assert t[0x07] == 7 * 2.0 ** -9              # largest subnormal
    assert t[0x38] == 1.0 and t[0xB8] == -1.0
    assert t[0x00] == 0.0 and math.copysign(1.0, t[0x80]) == -1.0
    assert math.isnan(t[0x7F]) and math.isnan(t[0xFF])
    assert np.isfinite(t).sum() == 254
    pos = t[:0x7F]
    assert np.all(np.diff(pos) > 0)              # codes order like values


def test_table_matches_torch_float8_e4m3fn():
    codes = torch.arange(256, dtype=torch.int32).to(torch.uint8)
    ref = codes.view(torch.float8_e4m3fn).to(torch.float64).numpy()
    ours = fp8.e4m3_table()
    np.testing.assert_array_equal(np.isnan(ref), np.isnan(ours))
    ok = ~np.isnan(ref)
    np.testing.assert_array_equal(ref[ok], ours[ok])


def test_encode_matches_torch_including_ties():
    g = np.random.default_rng(11)
    v = np.concatenate([
        g.uniform(-448, 448, 20000), g.standard_normal(20000), g.uniform(-2.0 ** -5, 2.0 ** -5, 20000),
        # exact midpoints between neighbouring values: the tie cases
        0.5 * (fp8.e4m3_table()[1:0x7E] + fp8.e4m3_table()[2:0x7F]),
        -0.5 * (fp8.e4m3_table()[0:0x7D] + fp8.e4m3_table()[1:0x7E]),
        [0.0, -0.0, 448.0, -448.0, 2.0 ** -10, -2.0 ** -10, 3 * 2.0 ** -11],
    ]).astype(np.float32)
    ref = torch.from_numpy(v).to(torch.float8_e4m3fn).view(torch.uint8).numpy()
    ours = fp8.e4m3_encode(v)
    np.testing.assert_array_equal(ours, ref)


def test_encode_is_nearest_with_even_ties():
    t = fp8.e4m3_table()
    mid = 0.5 * (t[0x38] + t[0x39])             # between 1.0 (even) and 1.125
    assert fp8.e4m3_encode([mid])[0] == 0x38
    mid = 0.5 * (t[0x39] + t[0x3A])             # between 1.125 and 1.25 (even)
    assert fp8.e4m3_encode([mid])[0] == 0x3A
    mid = 0.5 * (t[0x0F] + t[0x10])             # across a binade: to 0x10
    assert fp8.e4m3_encode([mid])[0] == 0x10
    assert fp8.e4m3_encode([2.0 ** -10])[0] == 0x00   # half the smallest subnormal: to zero (even)
    assert fp8.e4m3_encode([3 * 2.0 ** -10])[0] == 0x02
    g = np.random.default_rng(3)
    v = g.uniform(-448, 448, 5000)
    dec = t[fp8.e4m3_encode(v)]
    fin = t[np.isfinite(t)]
    best = np.min(np.abs(v[:, None] - fin[None, :]), axis=1)   # brute force
    np.testing.assert_array_equal(np.abs(v - dec), best)


def test_row_exponents_and_sk_couplings():
    from paper_2308_02329_amd import synth

    J = synth.sk_pm1(50, 50, 0).astype(np.float32)
    codes, expo = fp8.quantize(J)
    assert np.all(expo == 127 - 8)              # 1 <= 448 * 2^-8 = 1.75, 1 > 0.875
    np.testing.assert_array_equal(fp8.decode(codes, expo), J.astype(np.float64))
    G = synth.gaussian_j(64, 50, 1).astype(np.float32)
    codes, expo = fp8.quantize(G)
    e = expo.astype(int) - 127
    amax = np.abs(G).max(axis=1).astype(np.float64)
    assert np.all(amax <= 448 * 2.0 ** e) and np.all(amax > 448 * 2.0 ** (e - 1))
    dec = fp8.decode(codes, expo)
    # half a unit in the last place: 2^-4 relative above the subnormals, 2^-10 * 2^e below
    bound = np.maximum(np.abs(G) * 2.0 ** -4, 2.0 ** -10 * 2.0 ** e[:, None])
    assert np.all(np.abs(dec - G) <= bound)
    assert np.all(np.sign(dec) * np.sign(G) >= 0)


def test_degenerate_rows():
    J = np.zeros((3, 3), dtype=np.float32)
    J[1, 2] = np.inf
    J[2, 0] = 1e-45                             # needs e < -127
    codes, expo = fp8.quantize(J)
    assert expo[0] == 127 and np.all(codes[0] == 0)
    assert expo[1] == 0xFF and expo[2] == 0xFF
    assert np.isnan(fp8.decode(codes, expo)[1]).all()
