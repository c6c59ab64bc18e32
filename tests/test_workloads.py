"""The seeded generators: deterministic, per-channel, with the stated ranges."""
import numpy as np

import workloads as wl


def test_c1_deterministic_and_ranges():
    W1, X1 = wl.c1_channel(2)
    W2, X2 = wl.c1_channel(2)
    assert np.array_equal(W1, W2) and np.array_equal(X1, X2)
    assert W1.shape == (2, 128, 64) and X1.shape == (2, 64, 512)
    assert W1.dtype == np.float16 and X1.dtype == np.float16
    mag = np.hypot(W1[0].astype(float), W1[1].astype(float))
    assert np.all(np.abs(mag - 1) < 2e-3)
    assert X1.min() >= -127 and X1.max() <= 127
    assert np.all(X1 == np.rint(X1))
    assert not np.array_equal(wl.c1_channel(3)[1], X1)


def test_c2_weights_are_phasors_of_geometry():
    geo = wl.c2_geometry(K=16, M=8)
    W = wl.c2_weights(5, geo)
    ax, ay, bl, bm = geo
    assert np.all(np.hypot(ax, ay) <= 1000.0) and np.all(np.hypot(bl, bm) <= 0.05)
    f = wl.c2_frequency(5)
    phi = 2 * np.pi * f * (np.outer(bl, ax) + np.outer(bm, ay)) / wl.C0
    ref = np.exp(1j * phi)
    got = W[0].astype(float) + 1j * W[1].astype(float)
    assert np.max(np.abs(got - ref)) < 1e-3
    assert wl.c2_frequency(0) < wl.c2_frequency(255)


def test_bits_pad_cleared():
    g = wl.rng(9, 0, 0)
    w = wl.random_words(g, 5, 33)
    assert w.shape == (2, 5, 2)
    assert np.all(w[..., 1] >> np.uint32(1) == 0)


def test_c4_ranges():
    W, X = wl.c4_channel(M=64, K=32, N=8)
    assert X.min() >= -2048 and X.max() <= 2047
    assert W.shape == (2, 64, 32)
