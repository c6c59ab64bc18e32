"""Pins for the oracle's steering weights (Sec. II delay model, Eq. 3
weights): closed forms where the phase is a whole, half or quarter turn, and
the defining property of a steering vector: a plane wave arriving from a
beam's own direction sums coherently to K times its amplitude in that beam
(through the oracle's complex product), while other beams stay below K."""
import numpy as np

import oracle

C0 = 299792458.0


def test_broadside_and_origin_are_unit_weights():
    g = np.random.default_rng(0)
    pos = g.uniform(-500, 500, (40, 3))
    pos[7] = 0.0                                  # a sensor at the phase centre
    dirs = np.vstack([np.zeros(3), g.uniform(-0.1, 0.1, (5, 3))])  # beam 0: broadside
    w = oracle.steering_weights(pos, dirs, [150e6, 151e6], C0)
    assert np.array_equal(w[:, 0, :], np.ones((2, 40)))
    assert np.array_equal(w[:, :, 7], np.ones((2, 6)))


def test_whole_half_and_quarter_turns():
    """f s / c exactly 3, 2.5 and 1.25 cycles (dyadic values, exact in FP64)."""
    pos = np.array([[3.0, 0, 0], [2.5, 0, 0], [1.25, 0, 0], [0, 0, 0.5]])
    dirs = np.array([[1.0, 0, 0], [0, 0, 1.0]])
    w = oracle.steering_weights(pos, dirs, [1.0], 1.0)  # f = c = 1: cycles = s
    assert w[0, 0, 0] == 1.0
    assert w[0, 0, 1].real == -1.0 and abs(w[0, 0, 1].imag) < 1e-15
    assert abs(w[0, 0, 2].real) < 1e-15 and w[0, 0, 2].imag == 1.0
    assert w[0, 1, 3].real == -1.0 and abs(w[0, 1, 3].imag) < 1e-15  # z axis, half a cycle


def test_unit_modulus_and_periodicity():
    g = np.random.default_rng(1)
    pos = g.uniform(-1000, 1000, (64, 3))
    dirs = g.uniform(-0.05, 0.05, (32, 3))
    w = oracle.steering_weights(pos, dirs, [120e6], C0)
    assert np.allclose(np.abs(w), 1.0, atol=1e-15)
    # one wavelength further along the beam direction changes nothing
    lam = C0 / 120e6
    d = np.array([[0.6, 0.8, 0.0]])
    p0 = g.uniform(-100, 100, (16, 3))
    shift = p0 + 7 * lam * d
    a = oracle.steering_weights(p0, d, [120e6], C0)
    b = oracle.steering_weights(shift, d, [120e6], C0)
    assert np.allclose(a, b, atol=1e-9)


def test_plane_wave_sums_coherently_in_its_own_beam():
    """Sensor signals of a plane wave from direction u_j: x_k = A exp(-2 pi i f
    tau_k(u_j)) (the delayed narrowband signal of Eq. 1).  Beam j's weights undo
    exactly those delays, so B[j] = K A; the other beams are smaller."""
    g = np.random.default_rng(2)
    K, M, f = 96, 8, 150e6
    pos = np.column_stack([g.uniform(-300, 300, (K, 2)), np.zeros(K)])
    # well separated beams (0.02 apart in direction cosine, several beam widths)
    dirs = np.column_stack([(np.arange(M) - 3.5) * 0.02, np.zeros(M), np.zeros(M)])
    W = oracle.steering_weights(pos, dirs, [f], C0)[0]          # [M, K]
    A = 0.75 - 0.5j
    tau = pos @ dirs.T / C0                                      # [K, M] delays of each source direction
    X = A * np.exp(-2j * np.pi * f * tau)                        # column j: wave from beam j's direction
    B = oracle.cgemm(W[None], X[None])[0]                        # [M, M]
    assert np.allclose(np.diag(B), K * A, rtol=1e-9)
    off = np.abs(B[~np.eye(M, dtype=bool)])
    assert off.max() < 0.9 * K * abs(A)
