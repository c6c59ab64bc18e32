"""Pins for the FP8 (e4m3) parts of the oracle: the decode table against torch's
CPU float8_e4m3fn (an independent implementation), hand-derived values, and
the quantiser's rounding against torch's cast."""
import numpy as np
import pytest

import oracle

torch = pytest.importorskip("torch")


def test_decode_matches_torch_all_codes():
    codes = np.arange(256, dtype=np.uint8)
    ours = oracle.e4m3_decode(codes)
    ref = torch.from_numpy(codes).view(torch.float8_e4m3fn).float().numpy().astype(np.float64)
    nan = np.isnan(ref)
    assert np.array_equal(np.isnan(ours), nan)
    assert np.array_equal(ours[~nan], ref[~nan])


def test_decode_hand_values():
    d = oracle.e4m3_decode(np.array([0x00, 0x80, 0x38, 0x7E, 0xFE, 0x01, 0x08, 0x7F, 0x3C], np.uint8))
    assert d[0] == 0.0 and d[1] == 0.0 and np.signbit(d[1])
    assert d[2] == 1.0            # exponent 7, mantissa 0
    assert d[3] == 448.0 and d[4] == -448.0
    assert d[5] == 2.0 ** -9      # smallest subnormal
    assert d[6] == 2.0 ** -6      # smallest normal
    assert np.isnan(d[7])
    assert d[8] == 1.5


def test_quantiser_rounding_matches_torch_cast():
    """With amax = 448 the scale is 1 and the quantiser reduces to a plain
    nearest-even cast, which torch implements independently."""
    g = np.random.default_rng(0)
    v = np.concatenate([g.uniform(-448, 448, 4000), g.normal(0, 1e-2, 2000),
                        [448.0, -448.0, 0.0, 2.0 ** -10, 3 * 2.0 ** -10, 1.0625, 1.1875, 17.0, 19.0]])
    v = v.astype(np.float32)
    n = v.size + (v.size % 2)
    re = np.zeros((1, n // 2), np.float32)
    im = np.zeros((1, n // 2), np.float32)
    flat = np.zeros(n, np.float32)
    flat[:v.size] = v
    re[0] = flat[0::2]
    im[0] = flat[1::2]
    re[0, 0] = 448.0  # pin amax
    qr, qi, sc = oracle.quantize_e4m3_rows(re, im)
    assert sc[0] == 1.0
    ref_r = torch.from_numpy(re).to(torch.float8_e4m3fn).view(torch.uint8).numpy()
    ref_i = torch.from_numpy(im).to(torch.float8_e4m3fn).view(torch.uint8).numpy()
    assert np.array_equal(qr, ref_r) and np.array_equal(qi, ref_i)


def test_quantiser_scale_and_error_bound():
    g = np.random.default_rng(1)
    re = g.normal(0, 3.0, (50, 300)).astype(np.float32)
    im = g.normal(0, 3.0, (50, 300)).astype(np.float32)
    re[7] = 0.0
    im[7] = 0.0                        # all-zero row: scale 1, codes 0
    qr, qi, sc = oracle.quantize_e4m3_rows(re, im)
    amax = np.maximum(np.abs(re).max(1), np.abs(im).max(1))
    assert sc[7] == 1.0 and not qr[7].any() and not qi[7].any()
    rows = np.arange(50) != 7
    np.testing.assert_array_equal(sc[rows], (amax[rows] / np.float32(448.0)).astype(np.float32))
    dr = oracle.e4m3_decode(qr) * sc[:, None]
    di = oracle.e4m3_decode(qi) * sc[:, None]
    # e4m3 keeps 3 mantissa bits: relative rounding error <= 2^-4 for normals,
    # absolute error <= 2^-10 * scale in the subnormal range
    tol = np.maximum(np.abs(re) * 2.0 ** -4, 2.0 ** -10 * sc[:, None]) * (1 + 1e-6)
    assert np.all(np.abs(dr - re) <= tol)
    tol = np.maximum(np.abs(im) * 2.0 ** -4, 2.0 ** -10 * sc[:, None]) * (1 + 1e-6)
    assert np.all(np.abs(di - im) <= tol)
    # the element of largest magnitude maps to +-448 exactly
    big = np.maximum(np.abs(oracle.e4m3_decode(qr)).max(1), np.abs(oracle.e4m3_decode(qi)).max(1))
    assert np.all(big[rows] == 448.0)
