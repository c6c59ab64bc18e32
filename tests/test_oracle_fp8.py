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


@pytest.mark.parametrize("k", [-20, -7, -1, 1, 3, 12, 40])
def test_quantiser_at_power_of_two_scales_matches_torch_cast(k):
    """Rows whose largest magnitude is 448 * 2^k: the scale is exactly 2^k,
    and every code must equal torch's nearest-even cast of x * 2^-k (exact in
    fp32), ties and subnormals included -- the rule pinned away from unit
    scale, on an independent implementation of the rounding."""
    g = np.random.default_rng(100 + k)
    rows, cols = 24, 130
    base = np.concatenate([g.uniform(-448, 448, (rows, cols - 10)), g.normal(0, 1e-2, (rows, 10))], axis=1)
    base[:, :6] = [448.0, 1.0625, 1.1875, 17.0, 2.0 ** -10, 3 * 2.0 ** -10]  # ties and subnormals
    base[::2, 0] = -448.0
    re = np.ldexp(base, k).astype(np.float32)
    im = np.ldexp(np.roll(base, 3, axis=1) * 0.5, k).astype(np.float32)
    qr, qi, sc = oracle.quantize_e4m3_rows(re, im)
    assert np.all(sc == np.float32(np.ldexp(1.0, k)))
    for v, q in ((re, qr), (im, qi)):
        y = np.ldexp(v.astype(np.float64), -k).astype(np.float32)
        ref = torch.from_numpy(y).to(torch.float8_e4m3fn).view(torch.uint8).numpy()
        assert np.array_equal(q, ref)


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


# --------------------------------------------------------------------------
# per-32-block quantiser (power-of-two E8M0 scales)
# --------------------------------------------------------------------------

def test_block_exponent_hand_values():
    """amax 448 needs no scaling; just above it needs 2^1; 1.75 = 448 * 2^-8
    sits exactly on a boundary; an all-zero block gets 2^0."""
    cases = [(448.0, 0), (449.0, 1), (1.75, -8), (1.76, -7), (1.0, -8), (0.5, -9), (896.0, 1), (896.5, 2),
             (0.0, 0), (3.0e38, 120)]
    re = np.zeros((len(cases), 32), np.float32)
    im = np.zeros((len(cases), 32), np.float32)
    for r, (a, _) in enumerate(cases):
        im[r, 5] = -a  # the maximum may come from either part and either sign
    _, _, codes = oracle.quantize_e4m3_blocks(re, im)
    assert [int(c) - 127 for c in codes[:, 0]] == [e for _, e in cases]


def test_block_exponent_is_minimal():
    g = np.random.default_rng(4)
    mag = np.exp(g.uniform(-30, 30, (64, 96))).astype(np.float32)
    re = (mag * np.sign(g.normal(size=mag.shape))).astype(np.float32)
    im = np.roll(re, 7, axis=1)
    _, _, codes = oracle.quantize_e4m3_blocks(re, im)
    e = codes.astype(np.int64) - 127
    for b in range(3):
        blk = slice(32 * b, 32 * b + 32)
        amax = np.maximum(np.abs(re[:, blk]).max(1), np.abs(im[:, blk]).max(1)).astype(np.float64)
        assert np.all(amax <= 448.0 * np.ldexp(1.0, e[:, b]))
        assert np.all(amax > 448.0 * np.ldexp(1.0, e[:, b] - 1))


def test_block_codes_match_torch_cast():
    """Once the exponent is known the codes are a plain nearest-even cast of
    x * 2^-e, which torch implements independently.  cols = 77: a ragged last
    block of 13 receivers."""
    g = np.random.default_rng(5)
    re = (g.normal(0, 1, (40, 77)) * np.exp(g.uniform(-8, 8, (40, 1)))).astype(np.float32)
    im = (g.normal(0, 1, (40, 77)) * np.exp(g.uniform(-8, 8, (40, 1)))).astype(np.float32)
    re[3, 40:] = 0.0
    im[3, 40:] = 0.0  # an all-zero third block
    qr, qi, codes = oracle.quantize_e4m3_blocks(re, im)
    assert codes.shape == (40, 3) and codes[3, 2] == 127
    e = np.repeat(codes.astype(np.int64) - 127, 32, axis=1)[:, :77]
    for v, q in ((re, qr), (im, qi)):
        y = np.ldexp(v.astype(np.float64), -e).astype(np.float32)
        ref = torch.from_numpy(y).to(torch.float8_e4m3fn).view(torch.uint8).numpy()
        assert np.array_equal(q, ref)


def test_block_quantiser_error_bound():
    g = np.random.default_rng(6)
    re = g.normal(0, 50.0, (30, 128)).astype(np.float32)
    im = g.normal(0, 50.0, (30, 128)).astype(np.float32)
    qr, qi, codes = oracle.quantize_e4m3_blocks(re, im)
    s = np.repeat(oracle.e8m0_decode(codes), 32, axis=1)
    for v, q in ((re, qr), (im, qi)):
        d = oracle.e4m3_decode(q) * s
        tol = np.maximum(np.abs(v) * 2.0 ** -4, 2.0 ** -10 * s) * (1 + 1e-9)
        assert np.all(np.abs(d - v) <= tol)
