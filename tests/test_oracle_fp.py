"""Pins for the FP64 oracle of B[c] = W[c] X[c] (Eq. (3); complex product of
Sec. III-B).  Each test checks the oracle against something other than itself:
a hand-worked value, an independent library routine, or a closed form."""
import numpy as np
import pytest

import oracle
from workloads import planar_to_complex, random_f16_case


def test_hand_worked_example():
    # (1+2i)(3+4i) = 3 + 4i + 6i - 8 = -5 + 10i
    # (5+6i)(7+8i) = 35 + 40i + 42i - 48 = -13 + 82i ;  sum = -18 + 92i
    W = np.array([[[1 + 2j, 5 + 6j]]])
    X = np.array([[[3 + 4j], [7 + 8j]]])
    B = oracle.cgemm(W, X)
    assert B.shape == (1, 1, 1)
    assert B[0, 0, 0] == -18 + 92j
    # a conjugated weight would give (1-2i)(3+4i)+(5-6i)(7+8i) = 94 + 0i... not this
    assert oracle.cgemm(np.conj(W), X)[0, 0, 0] != B[0, 0, 0]


@pytest.mark.parametrize("batch,M,N,K", [(1, 1, 1, 1), (2, 3, 5, 7), (3, 17, 9, 33), (1, 40, 64, 8)])
def test_matches_numpy_matmul(batch, M, N, K):
    g = np.random.default_rng(7 + M + N + K)
    W = g.normal(size=(batch, M, K)) + 1j * g.normal(size=(batch, M, K))
    X = g.normal(size=(batch, K, N)) + 1j * g.normal(size=(batch, K, N))
    B = oracle.cgemm(W, X)
    ref = np.matmul(W, X)  # independent library routine (complex128)
    np.testing.assert_allclose(B, ref, rtol=1e-12, atol=1e-12 * K)


def test_shared_weights_broadcast():
    g = np.random.default_rng(3)
    W = g.normal(size=(6, 5)) + 1j * g.normal(size=(6, 5))
    X = g.normal(size=(4, 5, 3)) + 1j * g.normal(size=(4, 5, 3))
    B = oracle.cgemm(W, X)
    for c in range(4):
        np.testing.assert_allclose(B[c], W @ X[c], rtol=1e-12)


@pytest.mark.parametrize("K", [1, 4, 64, 576])
def test_plane_wave_on_own_beam_exact(K):
    """A plane wave x_k = a e^{-i theta_k} s_n steered with w_k = e^{+i theta_k}
    adds coherently: |B| = K a (Eq. (1)-(3)).  Quarter-turn phases make every
    value exact, so the sum is exact."""
    g = np.random.default_rng(K)
    q = g.integers(0, 4, K)
    a = 3.0
    w = (1j) ** q                      # e^{+i theta_k}, theta_k in {0, pi/2, pi, 3pi/2}
    s = (1j) ** g.integers(0, 4, 5)    # unit-modulus signal samples
    X = a * np.outer((1j) ** (-q), s)  # [K, N]
    others = np.exp(1j * g.uniform(0, 2 * np.pi, (3, K)))
    W = np.vstack([others[:1], w[None, :], others[1:]])
    B = oracle.cgemm(W[None], X[None])[0]
    np.testing.assert_array_equal(np.abs(B[1]), np.full(5, K * a))
    np.testing.assert_array_equal(B[1], K * a * s)


def test_plane_wave_general_angles():
    """Same closed form with arbitrary delays: |B| = K a up to FP64 rounding."""
    K, N = 300, 16
    g = np.random.default_rng(11)
    d = g.uniform(-500.0, 500.0, K)          # sensor positions (m)
    theta, f, c0 = 0.3, 150e6, 299792458.0
    tau = d * np.sin(theta) / c0             # Eq. (2)
    ph = 2 * np.pi * f * tau
    s = np.exp(1j * g.uniform(0, 2 * np.pi, N))
    X = 2.5 * np.outer(np.exp(-1j * ph), s)  # narrow-band Eq. (1), noise-free
    W = np.exp(1j * ph)[None, :]
    B = oracle.cgemm(W[None], X[None])[0, 0]
    np.testing.assert_allclose(np.abs(B), K * 2.5, rtol=1e-12)


@pytest.mark.parametrize("K", [4, 8, 64])
def test_orthogonal_phasors(K):
    """DFT rows against DFT columns: B = K delta_{m j}; off-beam outputs vanish."""
    k = np.arange(K)
    W = np.exp(-2j * np.pi * np.outer(k, k) / K)   # [M=K, K]
    X = np.exp(+2j * np.pi * np.outer(k, k) / K)   # [K, N=K], column j = e^{+2 pi i jk/K}
    B = oracle.cgemm(W[None], X[None])[0]
    np.testing.assert_allclose(B, K * np.eye(K), atol=1e-12 * K * K)
    if K == 4:  # entries +-1, +-i: exact
        W4 = (1j) ** (-(np.outer(k, k) % 4))
        X4 = (1j) ** (np.outer(k, k) % 4)
        np.testing.assert_array_equal(oracle.cgemm(W4[None], X4[None])[0], 4 * np.eye(4))


def test_real_special_case_reduces_to_real_gemm():
    g = np.random.default_rng(5)
    Wr = g.normal(size=(2, 7, 9))
    Xr = g.normal(size=(2, 9, 4))
    B = oracle.cgemm(Wr.astype(complex), Xr.astype(complex))
    np.testing.assert_allclose(B.real, np.matmul(Wr, Xr), rtol=1e-12, atol=1e-12)
    assert np.all(B.imag == 0)
    # purely imaginary times purely imaginary is real and negated
    B2 = oracle.cgemm(1j * Wr, 1j * Xr)
    np.testing.assert_allclose(B2.real, -np.matmul(Wr, Xr), rtol=1e-12, atol=1e-12)


def test_entries_and_abs_dot():
    W, X = random_f16_case(1, 3, 19, 23, 37)
    Wc, Xc = planar_to_complex(W), planar_to_complex(X)
    full = oracle.cgemm(Wc, Xc)
    g = np.random.default_rng(0)
    cs, ms, ns = g.integers(0, 3, 50), g.integers(0, 19, 50), g.integers(0, 23, 50)
    e = oracle.cgemm_entries(Wc, Xc, cs, ms, ns)
    np.testing.assert_array_equal(e, full[cs, ms, ns])
    ad = oracle.abs_dot_entries(Wc, Xc, cs, ms, ns)
    ref = np.einsum("sk,sk->s", np.abs(Wc[cs, ms, :]), np.abs(Xc[cs, :, ns]))
    np.testing.assert_allclose(ad, ref, rtol=1e-12)
    assert np.all(np.abs(e) <= ad * (1 + 1e-12))


def test_fp16_widening_is_exact():
    W, X = random_f16_case(2, 1, 4, 4, 4)
    Wc = planar_to_complex(W)
    assert np.all(Wc.real.astype(np.float16).astype(np.float64) == Wc.real)


def test_index_validation():
    W = np.ones((1, 2, 3), complex)
    X = np.ones((1, 3, 4), complex)
    with pytest.raises(ValueError):
        oracle.cgemm_entries(W, X, [0], [2], [0])
    with pytest.raises(ValueError):
        oracle.cgemm(np.ones((1, 2, 5)), X)
