"""GPU parity of the 1-bit mode (sign packing and the three GEMM variants)
against the int64 oracle, through the C ABI.  Every comparison is bit-exact.
Variant 3 (e2m1 matrix instructions) takes K <= 2^23 with a whole number of
16-byte chunks per packed row (ceil(K / 32) a multiple of 4); other shapes
must be refused by the plan."""
import numpy as np
import pytest

import oracle
import workloads as wl
from gpu_util import log, to_dev, words_to_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_2505_03269_amd as tcbf  # noqa: E402

VARIANTS = [1, 2, 3]


def fp4_accepts(K, M=1, N=1):
    kw = (K + 31) // 32
    return K <= (1 << 23) and kw % 4 == 0 and 8 * M * kw < 2**31 and 8 * N * kw < 2**31 and 8 * M * N < 2**31


def run_1bit(Wp, Xp, K, variant, c_layout=tcbf.PLANAR, shared=False):
    """Wp [nb,2,M,kw], Xp [batch,2,N,kw] uint32 -> int64 (Re, Im) [batch,M,N]."""
    batch, _, N, kw = Xp.shape
    M = Wp.shape[2]
    if variant == 3 and not fp4_accepts(K, M, N):
        with pytest.raises(tcbf.TcbfError):
            tcbf.Plan(batch, M, N, K, tcbf.INT1, c_layout=c_layout, a_shared=shared, variant=variant)
        pytest.skip("variant 3 refuses K=%d (checked)" % K)
    plan = tcbf.Plan(batch, M, N, K, tcbf.INT1, c_layout=c_layout, a_shared=shared, variant=variant)
    A, B = words_to_dev(Wp), words_to_dev(Xp)
    C = plan.empty_output()
    plan.execute(A, B, C)
    torch.cuda.synchronize()
    Ch = C.cpu().numpy().astype(np.int64)
    if c_layout == tcbf.PLANAR:
        return Ch[:, 0], Ch[:, 1]
    return Ch[..., 0], Ch[..., 1]


def oracle_1bit(Wp, Xp, K, shared=False):
    if shared:
        return oracle.cgemm_1bit_popc(Wp[0, 0], Wp[0, 1], Xp[:, 0], Xp[:, 1], K)
    return oracle.cgemm_1bit_popc(Wp[:, 0], Wp[:, 1], Xp[:, 0], Xp[:, 1], K)


SHAPES = [
    (1, 1, 1, 1), (1, 5, 7, 31), (2, 33, 17, 32), (1, 17, 33, 33), (1, 128, 128, 128), (2, 129, 65, 63),
    (1, 64, 64, 64), (1, 65, 64, 65), (1, 130, 257, 127), (1, 100, 100, 129), (1, 64, 200, 577),
    (1, 256, 130, 1000), (1, 70, 90, 8191), (1, 128, 128, 8192),
    (2, 129, 65, 100), (1, 130, 257, 511), (1, 17, 33, 1280), (1, 200, 136, 3060), (3, 64, 64, 2048),
]


@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("batch,M,N,K", SHAPES)
def test_gemm_bit_exact(variant, batch, M, N, K):
    log("1bit v%d: batch=%d M=%d N=%d K=%d" % (variant, batch, M, N, K))
    Wp, Xp = wl.random_bits_case(21, batch, M, N, K)
    gr, gi = run_1bit(Wp, Xp, K, variant)
    rr, ri = oracle_1bit(Wp, Xp, K)
    assert np.array_equal(gr, rr)
    assert np.array_equal(gi, ri)


@pytest.mark.parametrize("variant", VARIANTS)
def test_interleaved_output_and_shared(variant):
    K = 300 if variant != 3 else 490
    Wp, Xp = wl.random_bits_case(5, 3, 70, 50, K, shared_w=True)
    rr, ri = oracle_1bit(Wp, Xp, K, shared=True)
    gr, gi = run_1bit(Wp, Xp, K, variant, c_layout=tcbf.INTERLEAVED, shared=True)
    assert np.array_equal(gr, rr) and np.array_equal(gi, ri)


@pytest.mark.parametrize("variant", VARIANTS)
def test_nonzero_pad_bits_are_ignored(variant):
    """Bits past K in the last word do not affect the result."""
    K = 45 if variant != 3 else 109
    Wp, Xp = wl.random_bits_case(8, 1, 40, 40, K)
    rr, ri = oracle_1bit(Wp, Xp, K)
    Wd, Xd = Wp.copy(), Xp.copy()
    Wd[..., -1] |= np.uint32(0xFFFFE000)
    Xd[..., -1] |= np.uint32(0xABC00000)
    gr, gi = run_1bit(Wd, Xd, K, variant)
    assert np.array_equal(gr, rr) and np.array_equal(gi, ri)


def test_closed_forms():
    """Weight rows equal to the conjugate data column give Re = 2K, Im = 0;
    all (1+i) gives Re = 0, Im = 2K."""
    K, N = 200, 64
    g = np.random.default_rng(2)
    xr = g.choice([-1.0, 1.0], (N, K))
    xi = g.choice([-1.0, 1.0], (N, K))
    Xp = np.stack([oracle.pack1bit(xr), oracle.pack1bit(xi)])[None]        # [1,2,N,kw]
    Wp = np.stack([oracle.pack1bit(xr), oracle.pack1bit(-xi)])[None]       # row n = conj(column n)
    for v in VARIANTS:
        gr, gi = run_1bit(Wp, Xp, K, v)
        assert np.all(np.diag(gr[0]) == 2 * K) and np.all(np.diag(gi[0]) == 0)
        ones = np.stack([oracle.pack1bit(np.ones((N, K)))] * 2)[None]
        gr, gi = run_1bit(ones, ones, K, v)
        assert np.all(gr == 0) and np.all(gi == 2 * K)


# ---------------------------------------------------------------------------
# packing
# ---------------------------------------------------------------------------

def _src(g, dtype, shape):
    if dtype == np.int8:
        a = g.integers(-128, 128, shape).astype(np.int8)
        a.flat[::17] = 0
        return a
    a = g.normal(size=shape).astype(dtype)
    a.flat[::13] = 0.0
    a.flat[5::29] = -0.0
    return a


@pytest.mark.parametrize("dtype", [np.int8, np.float16, np.float32])
@pytest.mark.parametrize("k_major", [True, False])
@pytest.mark.parametrize("layout", [tcbf.PLANAR, tcbf.INTERLEAVED])
@pytest.mark.parametrize("K", [1, 31, 32, 33, 100, 129, 600])
@pytest.mark.parametrize("rows", [37, 64])
def test_pack_matches_oracle(dtype, k_major, layout, K, rows):
    """rows = 37 takes the per-row N-major kernel, rows = 64 the vectorised one."""
    g = np.random.default_rng(K)
    batch = 2
    if layout == tcbf.PLANAR:
        shape = (batch, 2, rows, K) if k_major else (batch, 2, K, rows)
    else:
        shape = (batch, rows, K, 2) if k_major else (batch, K, rows, 2)
    src = _src(g, dtype, shape)
    got = tcbf.pack1bit(to_dev(src), k_major=k_major, layout=layout)
    torch.cuda.synchronize()
    got = got.cpu().numpy().view(np.uint32)
    # oracle side: bring to [batch, 2, rows, K] values, then pack
    if layout == tcbf.PLANAR:
        v = src if k_major else np.swapaxes(src, 2, 3)
    else:
        v = np.moveaxis(src, 3, 1) if k_major else np.moveaxis(np.swapaxes(src, 1, 2), 3, 1)
    ref = oracle.pack1bit(v.astype(np.float64))
    assert np.array_equal(got, ref)


def test_pack_then_gemm_end_to_end():
    """int8 interleaved data [K][N][2] and K-major weights, packed on the GPU,
    then multiplied: equals the int64 definition on the signs."""
    g = np.random.default_rng(9)
    batch, M, N, K = 2, 96, 160, 250
    wsrc = g.integers(-128, 128, (batch, M, K, 2)).astype(np.int8)
    xsrc = g.integers(-128, 128, (batch, K, N, 2)).astype(np.int8)
    Wd = tcbf.pack1bit(to_dev(wsrc), k_major=True, layout=tcbf.INTERLEAVED)
    Xd = tcbf.pack1bit(to_dev(xsrc), k_major=False, layout=tcbf.INTERLEAVED)
    sgn = lambda a: np.where(a >= 0, 1, -1).astype(np.int8)  # noqa: E731
    rr, ri = oracle.cgemm_1bit_def(sgn(wsrc[..., 0]), sgn(wsrc[..., 1]), sgn(xsrc[..., 0]), sgn(xsrc[..., 1]))
    for v in VARIANTS:
        if v == 3 and not fp4_accepts(K, M, N):
            continue
        plan = tcbf.Plan(batch, M, N, K, tcbf.INT1, variant=v)
        C = plan.empty_output()
        plan.execute(Wd, Xd, C)
        torch.cuda.synchronize()
        Ch = C.cpu().numpy().astype(np.int64)
        assert np.array_equal(Ch[:, 0], rr) and np.array_equal(Ch[:, 1], ri)


# ---------------------------------------------------------------------------
# the one-bit workload at full size
# ---------------------------------------------------------------------------

def test_c3_full_size():
    """64 x 2048 x 8192 x 8192: channel 0 compared in full, plus 100k sampled
    entries over all channels (tile edges included), for the default plan."""
    cfg = wl.WORKLOADS["one-bit"]
    batch, M, N, K = cfg["batch"], cfg["M"], cfg["N"], cfg["K"]
    log("c3 full size: generating inputs")
    Wp, Xp = wl.generate_c3()
    plan = tcbf.Plan(batch, M, N, K, tcbf.INT1)
    A, B = words_to_dev(Wp), words_to_dev(Xp)
    C = plan.empty_output()
    log("c3 full size: execute variant %d" % plan.info()["variant"])
    plan.execute(A, B, C)
    torch.cuda.synchronize()
    c0 = C[0].cpu().numpy().astype(np.int64)
    log("c3: oracle channel 0")
    rr, ri = oracle.cgemm_1bit_popc(Wp[0:1, 0], Wp[0:1, 1], Xp[0:1, 0], Xp[0:1, 1], K)
    assert np.array_equal(c0[0], rr[0]) and np.array_equal(c0[1], ri[0])
    g = np.random.default_rng(77)
    cnt = 100000
    cs, ms, ns = g.integers(0, batch, cnt), g.integers(0, M, cnt), g.integers(0, N, cnt)
    em = np.array([0, 127, 128, M - 1]); en = np.array([0, 127, 128, N - 1])
    ec, emm, enn = np.meshgrid(np.arange(batch), em, en, indexing="ij")
    cs = np.concatenate([cs, ec.ravel()]); ms = np.concatenate([ms, emm.ravel()]); ns = np.concatenate([ns, enn.ravel()])
    idx = [torch.from_numpy(v).to("cuda:0") for v in (cs, ms, ns)]
    gr = C[idx[0], 0, idx[1], idx[2]].cpu().numpy().astype(np.int64)
    gi = C[idx[0], 1, idx[1], idx[2]].cpu().numpy().astype(np.int64)
    er, ei = oracle.cgemm_1bit_popc_entries(Wp[:, 0], Wp[:, 1], Xp[:, 0], Xp[:, 1], K, cs, ms, ns)
    assert np.array_equal(gr, er) and np.array_equal(gi, ei)


@pytest.mark.parametrize("variant", VARIANTS)
def test_longest_supported_k(variant):
    """K = 2^26 - 3 receivers (the library's limit is 2^26; a ragged last
    word): 32 x 32 outputs from random words, bit-exact against the oracle's
    popcount form on every output."""
    M = N = 32
    K = (1 << 26) - 3
    if variant == 3:
        # its own limit: 2^23 (exact fp32 sums); past it the plan refuses
        with pytest.raises(tcbf.TcbfError):
            tcbf.Plan(1, M, N, (1 << 23) + 128, tcbf.INT1, variant=3)
        K = 32 * 262140 - 3  # a ragged last word, and a last stage only partly inside K
    kw = (K + 31) // 32
    g = torch.Generator(device="cuda:0")
    g.manual_seed(41)
    log("1-bit K=%d variant %d" % (K, variant))
    A = torch.randint(-2**31, 2**31 - 1, (1, 2, M, kw), dtype=torch.int32, device="cuda:0", generator=g)
    B = torch.randint(-2**31, 2**31 - 1, (1, 2, N, kw), dtype=torch.int32, device="cuda:0", generator=g)
    mask = (1 << (K % 32)) - 1
    A[..., kw - 1] &= mask
    B[..., kw - 1] &= mask
    plan = tcbf.Plan(1, M, N, K, tcbf.INT1, variant=variant)
    C = plan.empty_output()
    plan.execute(A, B, C)
    torch.cuda.synchronize()
    Wp = A.cpu().numpy().view(np.uint32)
    Xp = B.cpu().numpy().view(np.uint32)
    rr, ri = oracle_1bit(Wp, Xp, K)
    Ch = C.cpu().numpy().astype(np.int64)
    assert np.array_equal(Ch[:, 0], rr) and np.array_equal(Ch[:, 1], ri)

