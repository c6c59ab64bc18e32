"""GPU parity of the FP16 mode against the FP64 oracle (through the C ABI).

Gate: relative Frobenius error <= 2e-3 per channel plus the per-element fp32
summation bound (see gpu_util).  Layout combinations must agree bitwise."""
import numpy as np
import pytest

import oracle
import workloads as wl
from gpu_util import (c_inter_to_complex, c_planar_to_complex, check_fp_entries, check_fp_full, gamma, log,
                      to_dev)

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_2505_03269_amd as tcbf  # noqa: E402


def run_f16(W, X, a_layout=tcbf.PLANAR, b_layout=tcbf.PLANAR, c_layout=tcbf.PLANAR, shared=False, variant=0):
    """W planar [nb,2,M,K], X planar [batch,2,K,N] (numpy fp16) -> complex128 [batch,M,N]."""
    batch, _, K, N = X.shape
    M = W.shape[2]
    plan = tcbf.Plan(batch, M, N, K, tcbf.F16, a_layout, b_layout, c_layout, a_shared=shared, variant=variant)
    Wd = W if a_layout == tcbf.PLANAR else np.ascontiguousarray(W.transpose(0, 2, 3, 1))
    Xd = X if b_layout == tcbf.PLANAR else np.ascontiguousarray(X.transpose(0, 2, 3, 1))
    A = to_dev(Wd)
    B = to_dev(Xd)
    C = plan.empty_output()
    plan.execute(A, B, C)
    torch.cuda.synchronize()
    Ch = C.cpu().numpy()
    return (c_planar_to_complex(Ch) if c_layout == tcbf.PLANAR else c_inter_to_complex(Ch)), Ch


def oracle_ref(W, X, shared=False):
    Wc = wl.planar_to_complex(W)
    Xc = wl.planar_to_complex(X)
    if shared:
        Wc = Wc[0]
    ref = oracle.cgemm(Wc, Xc)
    absdot = np.matmul(np.abs(Wc), np.abs(Xc))
    return ref, absdot


def test_c1_full_output():
    """The plain 4-channel workload (128 x 64 x 512), every output entry."""
    chans = [wl.c1_channel(c) for c in range(4)]
    W = np.stack([w for w, _ in chans])
    X = np.stack([x for _, x in chans])
    log("c1: batch=4 M=128 N=512 K=64")
    got, _ = run_f16(W, X)
    ref, absdot = oracle_ref(W, X)
    check_fp_full(got, ref, absdot, 64)


EDGE_SHAPES = [
    (1, 1, 1, 1), (1, 15, 17, 31), (2, 17, 15, 33), (1, 33, 129, 63), (3, 129, 33, 65),
    (1, 16, 16, 16), (1, 32, 32, 32), (2, 31, 1, 64), (1, 1, 31, 8), (1, 128, 128, 32),
    (1, 127, 256, 575), (1, 257, 130, 577), (2, 200, 64, 96), (1, 1000, 40, 24), (1, 64, 1000, 7),
]


@pytest.mark.parametrize("batch,M,N,K", EDGE_SHAPES)
def test_edge_shapes(batch, M, N, K):
    log("edge: batch=%d M=%d N=%d K=%d" % (batch, M, N, K))
    W, X = wl.random_f16_case(7, batch, M, N, K)
    got, _ = run_f16(W, X)
    ref, absdot = oracle_ref(W, X)
    check_fp_full(got, ref, absdot, K)


@pytest.mark.parametrize("batch,M,N,K", [(2, 70, 90, 45), (2, 128, 256, 64), (1, 33, 20, 12)])
def test_layouts_bitwise_identical(batch, M, N, K):
    W, X = wl.random_f16_case(11, batch, M, N, K)
    ref, absdot = oracle_ref(W, X)
    base, _ = run_f16(W, X)
    check_fp_full(base, ref, absdot, K)
    for al in (0, 1):
        for bl in (0, 1):
            for cl in (0, 1):
                log("layouts a=%d b=%d c=%d shape=%s" % (al, bl, cl, (batch, M, N, K)))
                got, _ = run_f16(W, X, al, bl, cl)
                assert np.array_equal(got, base), "layout (%d,%d,%d) differs from planar" % (al, bl, cl)


def test_batch_independence_and_determinism():
    W, X = wl.random_f16_case(3, 3, 150, 140, 100)
    full, _ = run_f16(W, X)
    again, _ = run_f16(W, X)
    assert np.array_equal(full, again)
    alone, _ = run_f16(W[1:2], X[1:2])
    assert np.array_equal(alone[0], full[1])


def test_shared_weights():
    W, X = wl.random_f16_case(4, 3, 96, 80, 40, shared_w=True)
    got, _ = run_f16(W, X, shared=True)
    ref, absdot = oracle_ref(W, X, shared=True)
    check_fp_full(got, ref, absdot, 40)


def test_plane_wave_exact():
    """Quarter-turn steering phases: the beam on the source sums coherently to
    exactly K * a; the GPU result must be exact."""
    K, N, M = 576, 256, 64
    g = np.random.default_rng(1)
    q = g.integers(0, 4, K)
    a = 3.0
    s = (1j) ** g.integers(0, 4, N)
    Xc = a * np.outer((1j) ** (-q), s)
    Wc = np.exp(1j * g.uniform(0, 2 * np.pi, (M, K)))
    Wc[5] = (1j) ** q
    W = np.stack([Wc.real, Wc.imag]).astype(np.float16)[None]
    X = np.stack([Xc.real, Xc.imag]).astype(np.float16)[None]
    got, _ = run_f16(W, X)
    np.testing.assert_array_equal(np.abs(got[0, 5]), np.full(N, K * a))


def test_orthogonal_phasors():
    for K in (4, 64):
        k = np.arange(K)
        Wc = np.exp(-2j * np.pi * np.outer(k, k) / K)
        Xc = np.exp(2j * np.pi * np.outer(k, k) / K)
        if K == 4:
            Wc = (1j) ** (-(np.outer(k, k) % 4))
            Xc = (1j) ** (np.outer(k, k) % 4)
        W = np.stack([Wc.real, Wc.imag]).astype(np.float16)[None]
        X = np.stack([Xc.real, Xc.imag]).astype(np.float16)[None]
        got, _ = run_f16(W, X)
        if K == 4:
            np.testing.assert_array_equal(got[0], 4 * np.eye(4))
        else:
            ref, absdot = oracle_ref(W, X)
            check_fp_full(got, ref, absdot, K)
            off = got[0] - np.diag(np.diag(got[0]))
            assert np.max(np.abs(off)) < 0.05 * K  # fp16-rounded phasors: leakage far below the beam


def _sample_indices(g, batch, M, N, count, tile=128):
    cs = g.integers(0, batch, count)
    ms = g.integers(0, M, count)
    ns = g.integers(0, N, count)
    # tile boundaries and corners, in every channel
    edge_m = np.unique(np.clip([0, tile - 1, tile, M // 2, M - tile, M - 1], 0, M - 1))
    edge_n = np.unique(np.clip([0, tile - 1, tile, N // 2, N - tile, N - 1], 0, N - 1))
    ec, em, en = np.meshgrid(np.arange(batch), edge_m, edge_n, indexing="ij")
    return (np.concatenate([cs, ec.ravel()]), np.concatenate([ms, em.ravel()]),
            np.concatenate([ns, en.ravel()]))


def _sampled_parity(W, X, C, K, shared=False, count=20000):
    batch, _, M, N = C.shape
    g = np.random.default_rng(123)
    cs, ms, ns = _sample_indices(g, batch, M, N, count)
    idx = [torch.from_numpy(v).to("cuda:0") for v in (cs, ms, ns)]
    gr = C[idx[0], 0, idx[1], idx[2]].cpu().numpy().astype(np.float64)
    gi = C[idx[0], 1, idx[1], idx[2]].cpu().numpy().astype(np.float64)
    got = gr + 1j * gi
    ref = np.empty(cs.size, complex)
    absdot = np.empty(cs.size)
    for c in np.unique(cs):
        sel = np.nonzero(cs == c)[0]
        Wc = wl.planar_to_complex(W[0 if shared else c])[None]
        Xc = wl.planar_to_complex(X[c])[None]
        z = np.zeros(sel.size, np.int64)
        ref[sel] = oracle.cgemm_entries(Wc, Xc, z, ms[sel], ns[sel])
        absdot[sel] = oracle.abs_dot_entries(Wc, Xc, z, ms[sel], ns[sel])
    check_fp_entries(got, ref, absdot, K)
    return got, ref


def test_c2_full_size_sampled():
    """The radio-astronomy workload at full size (256 x 1024 x 576 x 4096), the plan the
    benchmark times; 20k random entries plus tile edges of every channel."""
    cfg = wl.WORKLOADS["radio-astro-fp16"]
    log("c2 full size: generating inputs")
    W, X = wl.generate_c2()
    plan = tcbf.Plan(cfg["batch"], cfg["M"], cfg["N"], cfg["K"], tcbf.F16)
    A, B = to_dev(W), to_dev(X)
    C = plan.empty_output()
    log("c2 full size: execute")
    plan.execute(A, B, C)
    torch.cuda.synchronize()
    del A, B
    got, ref = _sampled_parity(W, X, C, cfg["K"])
    log("c2 sampled rel Frobenius %.3e" % (np.linalg.norm(got - ref) / np.linalg.norm(ref)))
    _full_output_sums(W, X, C, cfg["K"])


def _full_output_sums(W, X, C, K):
    """Every output entry, through two exact identities: the sum of a beam's
    row over all samples is W times the row sums of X, and the sum of a
    sample's column over all beams is the column sums of W times X (FP64
    oracle on the summed operands, which are exact in FP64).  The GPU sums
    are taken in FP64 on the device; the bound is the per-element fp32 bound
    summed over the row or column; a second, statistical gate takes 1e-6 of
    the sum's scale sum |w||x| (the worst-case bound is about 1e-4 of it and
    far from what rounding reaches: observed errors are below 1e-9 of the
    scale), so one output entry off by more than about a tenth of its own
    magnitude also shows.  Channel by channel on the host."""
    bound_f = 2.0 * gamma(2 * K)
    rows = C.sum(dim=3, dtype=torch.float64).cpu().numpy()       # [batch, 2, M]
    cols = C.sum(dim=2, dtype=torch.float64).cpu().numpy()       # [batch, 2, N]
    worst = {"row": 0.0, "column": 0.0}
    for c in range(W.shape[0]):
        Wc = W[c, 0].astype(np.float64) + 1j * W[c, 1].astype(np.float64)     # [M, K]
        Xc = X[c, 0].astype(np.float64) + 1j * X[c, 1].astype(np.float64)     # [K, N]
        aW, aX = np.abs(Wc), np.abs(Xc)
        ref_r = oracle.cgemm(Wc[None], Xc.sum(axis=1)[None, :, None])[0, :, 0]
        ref_c = oracle.cgemm(Wc.sum(axis=0)[None, None, :], Xc[None])[0, 0]
        bnd_r = bound_f * (aW @ aX.sum(axis=1))
        bnd_c = bound_f * (aW.sum(axis=0) @ aX)
        for got, ref, bnd, what in ((rows[c], ref_r, bnd_r, "row"), (cols[c], ref_c, bnd_c, "column")):
            err = np.maximum(np.abs(got[0] - ref.real), np.abs(got[1] - ref.imag))
            bad = err > bnd + 1e-9
            assert not bad.any(), "channel %d %s sums: %d outside the bound, worst %.3e vs %.3e" % (
                c, what, int(bad.sum()), float(err[bad].max()), float(bnd[bad].max()))
            scale = bnd / bound_f
            assert np.all(err <= 1e-6 * scale), "channel %d %s sums beyond 1e-6 of their scale" % (c, what)
            worst[what] = max(worst[what], float((err / scale).max()))
    log("c2 full-output sums: worst error / sum |w||x| %s" % worst)


def test_c4_full_size_sampled():
    """The ultrasound workload (1 x 32768 x 8192 x 256), fp16."""
    cfg = wl.WORKLOADS["ultrasound-fp16"]
    log("c4 full size: generating inputs")
    W, X = wl.c4_channel(0)
    W, X = W[None], X[None]
    plan = tcbf.Plan(1, cfg["M"], cfg["N"], cfg["K"], tcbf.F16)
    A, B = to_dev(W), to_dev(X)
    C = plan.empty_output()
    log("c4 full size: execute")
    plan.execute(A, B, C)
    torch.cuda.synchronize()
    del A, B
    got, ref = _sampled_parity(W, X, C, cfg["K"], count=5000)
    log("c4 sampled rel Frobenius %.3e" % (np.linalg.norm(got - ref) / np.linalg.norm(ref)))


def test_rejects_bad_tensors():
    plan = tcbf.Plan(1, 32, 32, 32, tcbf.F16)
    A = torch.zeros(plan.shape_a(), dtype=torch.float16, device="cuda:0")
    B = torch.zeros(plan.shape_b(), dtype=torch.float16, device="cuda:0")
    C = plan.empty_output()
    with pytest.raises(ValueError):
        plan.execute(A.float(), B, C)
    with pytest.raises(ValueError):
        plan.execute(A[..., :16], B, C)
    # misaligned pointer: rejected by the library itself
    flat = torch.zeros(A.numel() + 8, dtype=torch.float16, device="cuda:0")
    st = tcbf.lib().tcbf_execute(plan._h, flat.data_ptr() + 2, B.data_ptr(), C.data_ptr(), None, None, None)
    assert st == 1


ALIGNED_SHAPES = [(1, 1, 8, 8), (1, 130, 136, 40), (2, 200, 264, 72), (1, 129, 8, 520), (3, 64, 128, 32),
                  (1, 257, 392, 576), (2, 128, 128, 8), (1, 300, 264, 112)]


FAST_VARIANTS = [2, 3, 4, 5, 6, 7, 8, 9]


@pytest.mark.parametrize("batch,M,N,K", ALIGNED_SHAPES)
def test_fast_and_generic_kernels_agree_bitwise(batch, M, N, K):
    """Every fp16 kernel configuration feeds the matrix unit the same fragments
    in the same order: outputs must be identical, and within the gate."""
    W, X = wl.random_f16_case(13, batch, M, N, K)
    ref, absdot = oracle_ref(W, X)
    gen, _ = run_f16(W, X, variant=1)
    check_fp_full(gen, ref, absdot, K)
    for v in FAST_VARIANTS:
        log("variant %d: batch=%d M=%d N=%d K=%d" % (v, batch, M, N, K))
        fast, _ = run_f16(W, X, variant=v)
        assert np.array_equal(fast, gen), "variant %d differs from the generic kernel" % v
        fast_il, _ = run_f16(W, X, c_layout=tcbf.INTERLEAVED, variant=v)
        assert np.array_equal(fast_il, fast), "variant %d interleaved output differs" % v


def test_plan_picks_fast_kernel_for_aligned_planar():
    assert tcbf.Plan(256, 1024, 4096, 576, tcbf.F16).info()["variant"] >= 2
    assert tcbf.Plan(1, 64, 100, 64, tcbf.F16).info()["variant"] == 1          # N % 8 != 0
    assert tcbf.Plan(1, 64, 64, 64, tcbf.F16, a_layout=tcbf.INTERLEAVED).info()["variant"] == 1
    with pytest.raises(tcbf.TcbfError):
        tcbf.Plan(1, 64, 100, 64, tcbf.F16, variant=2)


def test_largest_channel_takes_the_generic_kernel():
    """A channel whose W plane pair is past the fast kernel's 2 GiB byte
    offsets (M = 32768 beams x K = 24576 receivers: 3.2 GB of fp16) but
    inside the 2^31-element planes the library supports: the plan falls back
    to the generic kernel, and small-integer data makes every sampled entry
    exact (all partial sums are integers below 2^24), so they must equal the
    oracle bit for bit -- beams past the 32-bit byte-offset range included."""
    M, N, K = 32768, 64, 24576
    plan = tcbf.Plan(1, M, N, K, tcbf.F16)
    assert plan.info()["kernel_name"] == "cgemm_f16_kernel"
    g = torch.Generator(device="cuda:0")
    g.manual_seed(31)
    log("largest channel: generating 3.2 GB of weights")
    A = torch.randint(-8, 9, plan.shape_a(), dtype=torch.float16, device="cuda:0", generator=g)
    B = torch.randint(-8, 9, plan.shape_b(), dtype=torch.float16, device="cuda:0", generator=g)
    C = plan.empty_output()
    plan.execute(A, B, C)
    torch.cuda.synchronize()
    rng = np.random.default_rng(32)
    ms = np.unique(np.concatenate([[0, M - 1, 21845, 21846], rng.integers(0, M, 60)]))
    ns = rng.integers(0, N, ms.size)
    ns[-1] = N - 1
    Wsub = A[:, :, torch.from_numpy(ms).cuda()].cpu().numpy().astype(np.float64)   # [1, 2, S, K]
    X = B.cpu().numpy().astype(np.float64)
    got = C.cpu().numpy()[0]
    Wc = Wsub[:, 0] + 1j * Wsub[:, 1]
    Xc = X[:, 0] + 1j * X[:, 1]
    ref = oracle.cgemm_entries(Wc, Xc, np.zeros(ms.size, np.int64), np.arange(ms.size), ns)
    assert np.array_equal(got[0, ms, ns], ref.real) and np.array_equal(got[1, ms, ns], ref.imag)



# interleaved data (X as [batch][K][N][2]) through the ping-pong kernel: small,
# ragged, multi-tile and long-K shapes (several 32-receiver stages, several
# tiles per workgroup)
IL_SHAPES = [(1, 130, 136, 40), (2, 200, 264, 72), (1, 129, 8, 520), (2, 1024, 1024, 576), (1, 300, 1000, 104),
             (1, 64, 4096, 2048)]


@pytest.mark.parametrize("batch,M,N,K", IL_SHAPES)
def test_interleaved_data_ping_pong_bitwise(batch, M, N, K):
    """Interleaved data through the ping-pong kernel (planar and receiver-blocked
    weights, planar and interleaved output) equals the generic kernel on
    planar data bit for bit, which passes the oracle gate."""
    W, X = wl.random_f16_case(17, batch, M, N, K)
    gen, _ = run_f16(W, X, variant=1)
    ref, absdot = oracle_ref(W, X)
    check_fp_full(gen, ref, absdot, K)
    Xi = to_dev(np.ascontiguousarray(X.transpose(0, 2, 3, 1)))
    for al in (tcbf.PLANAR, tcbf.BLOCKED):
        A = to_dev(W) if al == tcbf.PLANAR else tcbf.block_weights(to_dev(W))
        for cl in (tcbf.PLANAR, tcbf.INTERLEAVED):
            log("interleaved data: a=%d c=%d shape=%s" % (al, cl, (batch, M, N, K)))
            plan = tcbf.Plan(batch, M, N, K, tcbf.F16, a_layout=al, b_layout=tcbf.INTERLEAVED, c_layout=cl,
                             variant=9)
            C = plan.empty_output()
            plan.execute(A, Xi, C)
            torch.cuda.synchronize()
            Ch = C.cpu().numpy()
            got = c_planar_to_complex(Ch) if cl == tcbf.PLANAR else c_inter_to_complex(Ch)
            assert np.array_equal(got, gen), "interleaved data, a=%d c=%d differs" % (al, cl)


def test_interleaved_data_plan_choice():
    """Large interleaved-data problems take the ping-pong kernel; small ones the
    generic kernel, or the ping-pong kernel when W is receiver-blocked."""
    IL = tcbf.INTERLEAVED
    assert tcbf.Plan(256, 1024, 4096, 576, tcbf.F16, b_layout=IL).info()["variant"] == 9
    assert tcbf.Plan(256, 1024, 4096, 576, tcbf.F16, a_layout=tcbf.BLOCKED, b_layout=IL).info()["variant"] == 9
    assert tcbf.Plan(1, 64, 64, 64, tcbf.F16, b_layout=IL).info()["variant"] == 1
    assert tcbf.Plan(1, 64, 64, 64, tcbf.F16, a_layout=tcbf.BLOCKED, b_layout=IL).info()["variant"] == 9
    assert tcbf.Plan(1, 64, 100, 64, tcbf.F16, b_layout=IL).info()["variant"] == 1      # N % 8 != 0
    with pytest.raises(tcbf.TcbfError):
        tcbf.Plan(1, 64, 64, 64, tcbf.F16, b_layout=IL, variant=2)


def test_c2_full_size_interleaved_equals_planar():
    """The radio-astronomy workload at full size with interleaved data and
    interleaved output (weights receiver-blocked, the launch the benchmark's
    interleaved line times): the whole output equals the planar-data product bit
    for bit after de-interleaving (that product is checked against the oracle on
    sampled entries above)."""
    cfg = wl.WORKLOADS["radio-astro-fp16"]
    log("c2 interleaved: generating inputs")
    W, X = wl.generate_c2()
    A, B = to_dev(W), to_dev(X)
    del W, X
    Ab = tcbf.block_weights(A)
    del A
    Bi = B.permute(0, 2, 3, 1).contiguous()
    shape = (cfg["batch"], cfg["M"], cfg["N"], cfg["K"])
    pp = tcbf.Plan(*shape, tcbf.F16, a_layout=tcbf.BLOCKED)
    pi = tcbf.Plan(*shape, tcbf.F16, a_layout=tcbf.BLOCKED, b_layout=tcbf.INTERLEAVED, c_layout=tcbf.INTERLEAVED)
    assert pi.info()["variant"] == 9
    Cp = pp.empty_output()
    log("c2 interleaved: execute planar")
    pp.execute(Ab, B, Cp)
    del B
    Ci = pi.empty_output()
    log("c2 interleaved: execute interleaved")
    pi.execute(Ab, Bi, Ci)
    torch.cuda.synchronize()
    assert torch.equal(Cp, Ci.permute(0, 3, 1, 2))


def test_seeded_random_shapes_default_plan_and_variants():
    """Thirty seeded shapes (batch 1-5, M 1-700, N a multiple of 8 up to 520,
    K 1-1200; K a multiple of 8 in every other one so the fast kernels take
    them): the default plan (whichever kernel its rule picks) is within the
    gate against the oracle, and every variant that accepts the shape gives
    the default plan's output bit for bit."""
    rng = np.random.default_rng(77)
    for i in range(30):
        batch = int(rng.integers(1, 6))
        M = int(rng.integers(1, 701))
        N = 8 * int(rng.integers(1, 66))
        K = int(rng.integers(1, 1201))
        if i % 2 == 0:
            K = 8 * ((K + 7) // 8)
        W, X = wl.random_f16_case(1000 + i, batch, M, N, K)
        plan = tcbf.Plan(batch, M, N, K, tcbf.F16)
        log("random shape %d: %d x %d x %d x %d, default variant %d" % (i, batch, M, N, K, plan.info()["variant"]))
        got, _ = run_f16(W, X)
        ref, absdot = oracle_ref(W, X)
        check_fp_full(got, ref, absdot, K)
        for v in [1] + FAST_VARIANTS:
            try:
                tcbf.Plan(batch, M, N, K, tcbf.F16, variant=v)
            except tcbf.TcbfError:
                continue
            out, _ = run_f16(W, X, variant=v)
            assert np.array_equal(out, got), "shape %d: variant %d differs from the default plan" % (i, v)
