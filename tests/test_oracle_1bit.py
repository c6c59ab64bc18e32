"""Pins for the 1-bit oracle (Sec. III-D, Fig. 1, Table 2, the complex XOR
equations with padding, and the AND form of Sec. III-E).

The definition oracle (int64 sums of +-1 products) and the popcount oracle
(the paper's algorithm on packed words) are two independent routes; they are
checked against each other, against brute force in Python complex arithmetic,
against the paper's worked example and code table, and against closed forms."""
import itertools

import numpy as np
import pytest

import oracle
from conftest import read_golden
from workloads import random_bits_case


def _bits_display(words, K):
    """Bits in element order, first element first (the table's display order)."""
    return "".join(str((int(words[k // 32]) >> (k % 32)) & 1) for k in range(K))


def test_table2_worked_example():
    rows = read_golden("table2_dot1bit.txt")
    data = [r for r in rows if r[0] not in ("sum", "popc", "xorform")]
    summ = {r[0]: int(r[1]) for r in rows if r[0] in ("sum", "popc", "xorform")}
    A = np.array([int(r[0]) for r in data], np.float64)
    Bv = np.array([int(r[1]) for r in data], np.float64)
    prod = np.array([int(r[2]) for r in data])
    bA = "".join(r[3] for r in data)
    bB = "".join(r[4] for r in data)
    bX = "".join(r[5] for r in data)
    assert np.array_equal(A * Bv, prod)
    K = len(A)
    wa = oracle.pack1bit(A)
    wb = oracle.pack1bit(Bv)
    assert _bits_display(wa, K) == bA == "1010"
    assert _bits_display(wb, K) == bB == "1100"
    assert _bits_display(wa ^ wb, K) == bX
    assert bin(int(wa[0] ^ wb[0])).count("1") == summ["popc"]
    assert oracle.dot1bit_xor(wa, wb, K) == summ["xorform"] == summ["sum"] == int(prod.sum())
    assert oracle.dot1bit_and(wa, wb, K) == summ["sum"]


def test_fig1_code_table():
    for code, re, im in read_golden("fig1_codes.txt"):
        wr = np.array([int(code[0])], np.uint32)
        wi = np.array([int(code[1])], np.uint32)
        assert oracle.unpack1bit(wr, 1)[0] == int(re)
        assert oracle.unpack1bit(wi, 1)[0] == int(im)


def test_sign_rule_and_bit_order():
    v = np.array([0.0, -0.0, 1.0, -1.0, 5e-8, -7.0] + [1.0] * 26 + [-1.0, 2.0, -0.0])
    w = oracle.pack1bit(v)
    assert w.shape == (2,)
    # k=0 (+0) -> 1, k=1 (-0) -> 0, k=2 -> 1, k=3 -> 0, k=4 -> 1, k=5 -> 0, k=6..31 -> 1
    expect0 = 0b1 | (1 << 2) | (1 << 4) | sum(1 << k for k in range(6, 32))
    assert int(w[0]) == expect0
    assert int(w[1]) == 0b10  # k=32 -> 0, k=33 -> 1, k=34 (-0) -> 0, pad bits 0
    ints = np.array([0, -1, 1, -128, 127], np.float64)  # integer sources: 0 counts as +1
    assert int(oracle.pack1bit(ints)[0]) == 0b10101


@pytest.mark.parametrize("K", [1, 5, 31, 32, 33, 64, 100])
def test_pack_unpack_round_trip(K):
    g = np.random.default_rng(K)
    s = g.choice([-1, 1], size=(3, K)).astype(np.int8)
    w = oracle.pack1bit(s.astype(np.float64))
    assert w.shape == (3, oracle.words_per_row(K))
    np.testing.assert_array_equal(oracle.unpack1bit(w, K), s)
    if K % 32:
        assert np.all(w[:, -1] >> np.uint32(K % 32) == 0)  # pad bits are binary 0


def _all_vectors(K):
    """All 4^K vectors over {+-1 +-i}: planes [4^K, K] of +-1."""
    vals = [(r, i) for r in (-1, 1) for i in (-1, 1)]
    vecs = list(itertools.product(vals, repeat=K))
    re = np.array([[v[k][0] for k in range(K)] for v in vecs], np.int8)
    im = np.array([[v[k][1] for k in range(K)] for v in vecs], np.int8)
    return re, im


@pytest.mark.parametrize("K", [1, 2, 3])
def test_brute_force_all_small_vectors(K):
    re, im = _all_vectors(K)
    P = re.shape[0]
    # W rows: every vector; X columns: every vector
    Wr, Wi = re[None], im[None]                  # [1, P, K]
    Xr, Xi = re.T[None], im.T[None]              # [1, K, P]
    dr, di = oracle.cgemm_1bit_def(Wr, Wi, Xr, Xi)
    pr, pi = oracle.cgemm_1bit_popc(oracle.pack1bit(re.astype(float))[None],
                                    oracle.pack1bit(im.astype(float))[None],
                                    oracle.pack1bit(re.astype(float))[None],
                                    oracle.pack1bit(im.astype(float))[None], K)
    for a in range(P):
        for b in range(P):
            z = sum(complex(re[a, k], im[a, k]) * complex(re[b, k], im[b, k]) for k in range(K))
            assert (dr[0, a, b], di[0, a, b]) == (z.real, z.imag)
            assert (pr[0, a, b], pi[0, a, b]) == (z.real, z.imag)


@pytest.mark.parametrize("K", [31, 32, 33, 63, 64, 65, 100, 577])
def test_popcount_form_equals_definition(K):
    batch, M, N = 2, 5, 7
    Wp, Xp = random_bits_case(K, batch, M, N, K)
    Wr = oracle.unpack1bit(Wp[:, 0], K)
    Wi = oracle.unpack1bit(Wp[:, 1], K)
    Xr = np.swapaxes(oracle.unpack1bit(Xp[:, 0], K), 1, 2)
    Xi = np.swapaxes(oracle.unpack1bit(Xp[:, 1], K), 1, 2)
    dr, di = oracle.cgemm_1bit_def(Wr, Wi, Xr, Xi)
    pr, pi = oracle.cgemm_1bit_popc(Wp[:, 0], Wp[:, 1], Xp[:, 0], Xp[:, 1], K)
    np.testing.assert_array_equal(pr, dr)
    np.testing.assert_array_equal(pi, di)
    # entries variant
    cs = np.array([0, 1, 1]); ms = np.array([0, 4, 2]); ns = np.array([6, 0, 3])
    er, ei = oracle.cgemm_1bit_popc_entries(Wp[:, 0], Wp[:, 1], Xp[:, 0], Xp[:, 1], K, cs, ms, ns)
    np.testing.assert_array_equal(er, dr[cs, ms, ns])
    np.testing.assert_array_equal(ei, di[cs, ms, ns])
    # invariants: every +-1 complex product is 2 * {1, i, -1, -i}
    assert np.all(dr % 2 == 0) and np.all(di % 2 == 0)
    assert np.all(np.abs(dr) + np.abs(di) <= 2 * K)
    assert np.all((dr + di - 2 * K) % 4 == 0)


def test_unpadded_reading_of_K_is_wrong():
    """With K_pad > 0, reading the complex equations' K as the true K shifts Re
    by 2 K_pad; the padded reading (K_p) is the one that matches the sum."""
    K = 33
    Wp, Xp = random_bits_case(99, 1, 3, 3, K)
    pr, _ = oracle.cgemm_1bit_popc(Wp[:, 0], Wp[:, 1], Xp[:, 0], Xp[:, 1], K)
    Wr = oracle.unpack1bit(Wp[:, 0], K); Wi = oracle.unpack1bit(Wp[:, 1], K)
    Xr = np.swapaxes(oracle.unpack1bit(Xp[:, 0], K), 1, 2)
    Xi = np.swapaxes(oracle.unpack1bit(Xp[:, 1], K), 1, 2)
    dr, _ = oracle.cgemm_1bit_def(Wr, Wi, Xr, Xi)
    kpad = 64 - K
    np.testing.assert_array_equal(pr, dr)
    assert np.all(pr - 2 * kpad != dr)


@pytest.mark.parametrize("K", [1, 31, 32, 33, 200])
def test_closed_forms(K):
    g = np.random.default_rng(K + 1)
    xr = g.choice([-1, 1], K).astype(np.int8)
    xi = g.choice([-1, 1], K).astype(np.int8)
    # weight row = conjugate of the data column: every term is |x_k|^2 = 2
    Wr, Wi = xr[None, None, :], (-xi)[None, None, :]
    Xr, Xi = xr[None, :, None], xi[None, :, None]
    dr, di = oracle.cgemm_1bit_def(Wr, Wi, Xr, Xi)
    assert (dr[0, 0, 0], di[0, 0, 0]) == (2 * K, 0)
    pk = lambda v: oracle.pack1bit(v.astype(float))[None, None, :]  # noqa: E731
    pr, pi = oracle.cgemm_1bit_popc(pk(xr), pk(-xi), pk(xr), pk(xi), K)
    assert (pr[0, 0, 0], pi[0, 0, 0]) == (2 * K, 0)
    # all (1+i) times all (1+i): (1+i)^2 = 2i per term
    ones = np.ones(K, np.int8)
    pr, pi = oracle.cgemm_1bit_popc(pk(ones), pk(ones), pk(ones), pk(ones), K)
    assert (pr[0, 0, 0], pi[0, 0, 0]) == (0, 2 * K)
    # all (-1-i) words are zero words: same product 2i per term
    z = -ones
    pr, pi = oracle.cgemm_1bit_popc(pk(z), pk(z), pk(z), pk(z), K)
    assert (pr[0, 0, 0], pi[0, 0, 0]) == (0, 2 * K)


@pytest.mark.parametrize("L", [1, 4, 31, 32, 33, 95, 256])
def test_and_form_equals_xor_form(L):
    g = np.random.default_rng(L)
    for _ in range(20):
        a = g.choice([-1.0, 1.0], L)
        b = g.choice([-1.0, 1.0], L)
        wa, wb = oracle.pack1bit(a), oracle.pack1bit(b)
        ref = int(np.dot(a, b))
        assert oracle.dot1bit_xor(wa, wb, L) == ref
        assert oracle.dot1bit_and(wa, wb, L) == ref


def test_shared_weight_packed():
    K = 70
    Wp, Xp = random_bits_case(5, 3, 4, 6, K, shared_w=True)
    pr, pi = oracle.cgemm_1bit_popc(Wp[0, 0], Wp[0, 1], Xp[:, 0], Xp[:, 1], K)
    for c in range(3):
        r1, i1 = oracle.cgemm_1bit_popc(Wp[0, 0][None], Wp[0, 1][None], Xp[c:c + 1, 0], Xp[c:c + 1, 1], K)
        np.testing.assert_array_equal(pr[c], r1[0])
        np.testing.assert_array_equal(pi[c], i1[0])
