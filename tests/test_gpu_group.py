"""Grouped persistent launch (tcbf_group_execute) and HIP-graph capture.

The grouped kernel runs the same tile code as the plain fast kernel, so every
problem's output must equal its own single plan's output bit for bit, whatever
else shares the launch; one problem is also checked against the FP64 oracle.
Graph tests capture launches, replay them several times with eager work and
synchronisations between replays, and compare every replay with the eager
result."""
import numpy as np
import pytest

import oracle
import workloads as wl
from gpu_util import check_fp_full, log, to_dev, words_to_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_2505_03269_amd as tcbf  # noqa: E402

# (batch, M, N, K, shared W): uneven shapes, ragged tiles, one shared-W problem
MIX = [(1, 300, 264, 576), (2, 128, 128, 64), (1, 1000, 40, 8), (3, 200, 392, 200), (1, 64, 1024, 2048),
       (2, 513, 136, 96), (4, 96, 256, 576), (1, 130, 8, 1032)]


def make(seed, batch, M, N, K, shared=False, layout=tcbf.PLANAR):
    W, X = wl.random_f16_case(seed, batch, M, N, K, shared_w=shared)
    Cshape = (batch, 2, M, N) if layout == tcbf.PLANAR else (batch, M, N, 2)
    return W, X, to_dev(W), to_dev(X), torch.full(Cshape, float("nan"), device="cuda:0")


def single(Wd, Xd, batch, M, N, K, shared=False, layout=tcbf.PLANAR):
    plan = tcbf.Plan(batch, M, N, K, tcbf.F16, c_layout=layout, a_shared=shared)
    C = plan.empty_output()
    plan.execute(Wd, Xd, C)
    return C


@pytest.mark.parametrize("layout", [tcbf.PLANAR, tcbf.INTERLEAVED])
def test_group_equals_single_plans(layout):
    cases = []
    for i, (b, M, N, K) in enumerate(MIX):
        shared = i == 3
        cases.append((b, M, N, K, shared) + make(40 + i, b, M, N, K, shared, layout))
    log("group of %d problems, layout %d" % (len(cases), layout))
    tcbf.group_execute([(c[7], c[8], c[9], c[4]) for c in cases], c_layout=layout)
    torch.cuda.synchronize()
    for (b, M, N, K, shared, W, X, Wd, Xd, C) in cases:
        ref = single(Wd, Xd, b, M, N, K, shared, layout)
        torch.cuda.synchronize()
        got = C.cpu().numpy()
        assert not np.isnan(got).any(), (b, M, N, K)
        assert np.array_equal(got, ref.cpu().numpy()), (b, M, N, K)
    # and one against the oracle
    b, M, N, K, shared, W, X, Wd, Xd, C = cases[0]
    Ch = C.cpu().numpy().astype(np.float64)
    got = Ch[:, 0] + 1j * Ch[:, 1] if layout == tcbf.PLANAR else Ch[..., 0] + 1j * Ch[..., 1]
    Wc, Xc = wl.planar_to_complex(W), wl.planar_to_complex(X)
    check_fp_full(got, oracle.cgemm(Wc, Xc), np.matmul(np.abs(Wc), np.abs(Xc)), K)


def test_group_single_problem_and_full_list():
    """One problem alone, and a list of GROUP_MAX small problems."""
    b, M, N, K = 2, 256, 256, 128
    W, X, Wd, Xd, C = make(60, b, M, N, K)
    tcbf.group_execute([(Wd, Xd, C)])
    ref = single(Wd, Xd, b, M, N, K)
    torch.cuda.synchronize()
    assert np.array_equal(C.cpu().numpy(), ref.cpu().numpy())
    probs, refs = [], []
    for i in range(tcbf.GROUP_MAX):
        M, N, K = 8 + 8 * i, 16 + 8 * (i % 5), 8 * (1 + i % 7)
        W, X, Wd, Xd, C = make(70 + i, 1, M, N, K)
        probs.append((Wd, Xd, C))
        refs.append(single(Wd, Xd, 1, M, N, K))
    tcbf.group_execute(probs)
    torch.cuda.synchronize()
    for (Wd, Xd, C), r in zip(probs, refs):
        assert np.array_equal(C.cpu().numpy(), r.cpu().numpy())


def test_graph_capture_replays_match_eager():
    """Capture a grouped launch and a plain launch in one graph; change the
    inputs eagerly between replays; every replay must equal an eager run on
    the current inputs."""
    shapes = [(2, 200, 264, 576), (1, 96, 128, 64), (3, 128, 136, 200)]
    cases = [make(80 + i, *s) for i, s in enumerate(shapes)]
    W1, X1, Wd1, Xd1, _ = make(90, 2, 130, 128, 96)
    plan = tcbf.Plan(2, 130, 128, 96, tcbf.F16)
    C1 = plan.empty_output()
    ws = torch.empty(tcbf.GROUP_WORKSPACE_BYTES, dtype=torch.uint8, device="cuda:0")
    probs = [(c[2], c[3], c[4]) for c in cases]
    # warm up outside the capture, then capture on a side stream
    tcbf.group_execute(probs, workspace=ws)
    plan.execute(Wd1, Xd1, C1)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            tcbf.group_execute(probs, workspace=ws)
            plan.execute(Wd1, Xd1, C1)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    gen = torch.Generator(device="cuda:0")
    gen.manual_seed(5)
    for rep in range(4):
        # eager work between replays: new input values in the same buffers
        for (_, _, Wd, Xd, _) in cases + [(None, None, Wd1, Xd1, None)]:
            Xd.copy_(torch.randint(-127, 128, Xd.shape, device="cuda:0", generator=gen).half())
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for (W, X, Wd, Xd, C), (b, M, N, K) in zip(cases, shapes):
            ref = single(Wd, Xd, b, M, N, K)
            torch.cuda.synchronize()
            assert np.array_equal(C.cpu().numpy(), ref.cpu().numpy()), "replay %d" % rep
        ref1 = single(Wd1, Xd1, 2, 130, 128, 96)
        torch.cuda.synchronize()
        assert np.array_equal(C1.cpu().numpy(), ref1.cpu().numpy()), "replay %d" % rep


def test_group_rejects_bad_problems():
    W, X, Wd, Xd, C = make(99, 1, 64, 64, 64)
    with pytest.raises(ValueError):
        tcbf.group_execute([])
    with pytest.raises(ValueError):
        tcbf.group_execute([(Wd, Xd, C[:, :, :32])])
    W2, X2, Wd2, Xd2, C2 = make(98, 1, 64, 60, 64)       # N not a multiple of 8
    with pytest.raises(tcbf.TcbfError):
        tcbf.group_execute([(Wd2, Xd2, C2)])


# FP8: (batch, M, N, K, shared W) -- ragged K (K % 64 == 32 for the per-block
# tail), N a multiple of 4 but not of 8, one shared-W problem
F8_MIX = [(1, 300, 264, 576), (2, 128, 132, 96), (1, 1000, 40, 8), (3, 200, 392, 200), (1, 64, 1024, 2048),
          (2, 513, 136, 160), (1, 130, 8, 1032)]


def make_f8(seed, batch, M, N, K, dtype, shared=False, layout=tcbf.PLANAR):
    W, X = wl.random_f16_case(seed, batch, M, N, K, shared_w=shared)
    block = 0 if dtype == tcbf.F8_E4M3 else 32
    Wq, Ws = tcbf.quantize_e4m3(to_dev(W), k_major=True, block=block)
    Xq, Xs = tcbf.quantize_e4m3(to_dev(X), k_major=False, block=block)
    Cshape = (batch, 2, M, N) if layout == tcbf.PLANAR else (batch, M, N, 2)
    return Wq, Ws, Xq, Xs, torch.full(Cshape, float("nan"), device="cuda:0")


def single_f8(Wq, Ws, Xq, Xs, batch, M, N, K, dtype, shared=False, layout=tcbf.PLANAR):
    plan = tcbf.Plan(batch, M, N, K, dtype, c_layout=layout, a_shared=shared)
    C = plan.empty_output()
    plan.execute(Wq, Xq, C, Ws, Xs)
    return C


@pytest.mark.parametrize("layout", [tcbf.PLANAR, tcbf.INTERLEAVED])
@pytest.mark.parametrize("dtype", [tcbf.F8_E4M3, tcbf.MXF8_E4M3])
def test_group_f8_equals_single_plans(dtype, layout):
    cases = []
    for i, (b, M, N, K) in enumerate(F8_MIX):
        shared = i == 3
        cases.append(((b, M, N, K, shared), make_f8(140 + i, b, M, N, K, dtype, shared, layout)))
    log("fp8 group dtype %d layout %d" % (dtype, layout))
    tcbf.group_execute([(Wq, Xq, C, Ws, Xs, sh) for (_, _, _, _, sh), (Wq, Ws, Xq, Xs, C) in cases],
                       c_layout=layout, dtype=dtype)
    torch.cuda.synchronize()
    for (b, M, N, K, sh), (Wq, Ws, Xq, Xs, C) in cases:
        ref = single_f8(Wq, Ws, Xq, Xs, b, M, N, K, dtype, sh, layout)
        torch.cuda.synchronize()
        got = C.cpu().numpy()
        assert not np.isnan(got).any(), (b, M, N, K)
        assert np.array_equal(got, ref.cpu().numpy()), (dtype, b, M, N, K)


def test_group_f8_graph_replays_match_eager():
    """A captured grouped FP8 launch (per-block scales) replayed with new
    inputs quantised eagerly between replays equals single plans each time."""
    dtype = tcbf.MXF8_E4M3
    shapes = [(2, 200, 264, 576), (1, 96, 128, 96), (3, 128, 136, 200)]
    cases = [make_f8(160 + i, *s, dtype) for i, s in enumerate(shapes)]
    ws = torch.empty(tcbf.GROUP_WORKSPACE_BYTES, dtype=torch.uint8, device="cuda:0")
    probs = [(Wq, Xq, C, Ws, Xs) for (Wq, Ws, Xq, Xs, C) in cases]
    tcbf.group_execute(probs, workspace=ws, dtype=dtype)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            tcbf.group_execute(probs, workspace=ws, dtype=dtype)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    gen = torch.Generator(device="cuda:0")
    gen.manual_seed(7)
    for rep in range(3):
        for (Wq, Ws, Xq, Xs, C), (b, M, N, K) in zip(cases, shapes):
            X = torch.randint(-127, 128, (b, 2, K, N), device="cuda:0", generator=gen).half()
            tcbf.quantize_e4m3(X, k_major=False, block=32, out=Xq, scales=Xs)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for (Wq, Ws, Xq, Xs, C), (b, M, N, K) in zip(cases, shapes):
            ref = single_f8(Wq, Ws, Xq, Xs, b, M, N, K, dtype)
            torch.cuda.synchronize()
            assert np.array_equal(C.cpu().numpy(), ref.cpu().numpy()), "replay %d" % rep


def test_group_f8_rejects_mismatched_scales():
    Wq, Ws, Xq, Xs, C = make_f8(170, 1, 64, 64, 64, tcbf.F8_E4M3)
    with pytest.raises(ValueError):
        tcbf.group_execute([(Wq, Xq, C, Ws[:, :32], Xs)], dtype=tcbf.F8_E4M3)
    with pytest.raises(ValueError):
        tcbf.group_execute([(Wq, Xq, C, Ws, Xs)], dtype=tcbf.MXF8_E4M3)


# 1-bit: ragged K (partial last word, word counts not a multiple of 4), one
# shared-W problem, tiles cut by M and N
INT1_MIX = [(1, 300, 264, 576), (2, 128, 130, 95), (1, 1000, 40, 8), (3, 200, 392, 200), (1, 64, 1024, 2049),
            (2, 513, 136, 160), (1, 130, 8, 1032)]


@pytest.mark.parametrize("layout", [tcbf.PLANAR, tcbf.INTERLEAVED])
def test_group_int1_equals_single_plans_and_oracle(layout):
    cases = []
    for i, (b, M, N, K) in enumerate(INT1_MIX):
        shared = i == 3
        Wp, Xp = wl.random_bits_case(180 + i, b, M, N, K, shared_w=shared)
        Cshape = (b, 2, M, N) if layout == tcbf.PLANAR else (b, M, N, 2)
        C = torch.full(Cshape, -7, dtype=torch.int32, device="cuda:0")
        cases.append(((b, M, N, K, shared), Wp, Xp, words_to_dev(Wp), words_to_dev(Xp), C))
    log("1-bit group layout %d" % layout)
    tcbf.group_execute([(Wd, Xd, C, K, sh) for (_, _, _, K, sh), _, _, Wd, Xd, C in cases], c_layout=layout,
                       dtype=tcbf.INT1)
    torch.cuda.synchronize()
    for (b, M, N, K, sh), Wp, Xp, Wd, Xd, C in cases:
        plan = tcbf.Plan(b, M, N, K, tcbf.INT1, c_layout=layout, a_shared=sh, variant=1)
        ref = plan.empty_output()
        plan.execute(Wd, Xd, ref)
        torch.cuda.synchronize()
        got = C.cpu().numpy()
        assert np.array_equal(got, ref.cpu().numpy()), (b, M, N, K)
        Wr, Wi = (Wp[0, 0], Wp[0, 1]) if sh else (Wp[:, 0], Wp[:, 1])
        rr, ri = oracle.cgemm_1bit_popc(Wr, Wi, Xp[:, 0], Xp[:, 1], K)
        g64 = got.astype(np.int64)
        gr, gi = (g64[:, 0], g64[:, 1]) if layout == tcbf.PLANAR else (g64[..., 0], g64[..., 1])
        assert np.array_equal(gr, rr) and np.array_equal(gi, ri), (b, M, N, K)



# --------------------------------------------------------------------------
# receiver-blocked operands in a grouped launch
# --------------------------------------------------------------------------

MIX_BLOCKED = MIX + [(2, 200, 136, 100), (1, 70, 64, 7)]  # receiver counts that are not multiples of 8


@pytest.mark.parametrize("layout", [tcbf.PLANAR, tcbf.INTERLEAVED])
def test_group_blocked_weights_equal_single_plans(layout):
    """fp16 with receiver-blocked W: every problem equals its planar single
    plan's output bit for bit (blocked single plans where K is not a multiple
    of 8, which planar W cannot take on the fast path)."""
    cases = []
    for i, (b, M, N, K) in enumerate(MIX_BLOCKED):
        shared = i == 3
        W, X, Wd, Xd, C = make(60 + i, b, M, N, K, shared, layout)
        cases.append((b, M, N, K, shared, Wd, tcbf.block_weights(Wd), Xd, C))
    log("blocked group of %d problems, layout %d" % (len(cases), layout))
    tcbf.group_execute([(c[6], c[7], c[8], c[4]) for c in cases], c_layout=layout, layout=tcbf.BLOCKED)
    torch.cuda.synchronize()
    for (b, M, N, K, shared, Wd, Wb, Xd, C) in cases:
        if K % 8 == 0:
            ref = single(Wd, Xd, b, M, N, K, shared, layout)
        else:
            plan = tcbf.Plan(b, M, N, K, tcbf.F16, a_layout=tcbf.BLOCKED, c_layout=layout, a_shared=shared)
            ref = plan.empty_output()
            plan.execute(Wb, Xd, ref)
        torch.cuda.synchronize()
        got = C.cpu().numpy()
        assert not np.isnan(got).any(), (b, M, N, K)
        assert np.array_equal(got, ref.cpu().numpy()), (b, M, N, K)


@pytest.mark.parametrize("dtype", [tcbf.F8_E4M3, tcbf.MXF8_E4M3])
def test_group_f8_blocked_codes_equal_single_plans(dtype):
    """FP8 with receiver-blocked codes (the quantiser writes them): every
    problem equals its row-major single plan's output bit for bit."""
    block = 0 if dtype == tcbf.F8_E4M3 else 32
    BL = tcbf.BLOCKED
    cases = []
    for i, (b, M, N, K) in enumerate(MIX + [(2, 70, 36, 40), (1, 64, 64, 100)]):
        shared = i == 3
        nw = 1 if shared else b
        W = to_dev(wl.random_f16_case(80 + i, nw, M, 8, K)[0])
        X = to_dev(wl.random_f16_case(90 + i, b, 8, N, K)[1])
        pw, px = tcbf.quantize_e4m3(W, k_major=True, block=block), tcbf.quantize_e4m3(X, k_major=False, block=block)
        bw = tcbf.quantize_e4m3(W, k_major=True, block=block, out_layout=BL)
        bx = tcbf.quantize_e4m3(X, k_major=False, block=block, out_layout=BL)
        C = torch.full((b, 2, M, N), float("nan"), device="cuda:0")
        cases.append((b, M, N, K, shared, pw, px, bw, bx, C))
    log("blocked f8 group dtype %d: %d problems" % (dtype, len(cases)))
    tcbf.group_execute([(c[7][0], c[8][0], c[9], c[7][1], c[8][1], c[3], c[4]) for c in cases], dtype=dtype,
                       layout=BL)
    torch.cuda.synchronize()
    for (b, M, N, K, shared, pw, px, bw, bx, C) in cases:
        plan = tcbf.Plan(b, M, N, K, dtype, a_shared=shared)
        ref = plan.empty_output()
        plan.execute(pw[0], px[0], ref, pw[1], px[1])
        torch.cuda.synchronize()
        got = C.cpu().numpy()
        assert not np.isnan(got).any(), (b, M, N, K)
        assert np.array_equal(got, ref.cpu().numpy()), (b, M, N, K)


def test_group_blocked_graph_replays_match_eager():
    """A captured blocked-weight grouped launch replays to the eager result."""
    cases = []
    for i, (b, M, N, K) in enumerate(MIX[:4]):
        W, X, Wd, Xd, C = make(100 + i, b, M, N, K)
        cases.append((tcbf.block_weights(Wd), Xd, C))
    ws = torch.zeros(tcbf.GROUP_WORKSPACE_BYTES, dtype=torch.uint8, device="cuda:0")
    probs = [(a, x, c) for a, x, c in cases]
    tcbf.group_execute(probs, workspace=ws, layout=tcbf.BLOCKED)
    torch.cuda.synchronize()
    eager = [c.clone() for _, _, c in cases]
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            tcbf.group_execute(probs, workspace=ws, layout=tcbf.BLOCKED, stream=s)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    for r in range(3):
        for _, _, c in cases:
            c.fill_(float("nan"))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for c, e in zip([c for _, _, c in cases], eager):
            assert torch.equal(c, e), "replay %d differs" % r


# per-problem variants: 256-beam-tile variants (6, 7, 9) run in the grouped
# ping-pong launch, the rest in the grouped 128 x 128 launch
PP_VARIANTS = [9, 2, 9, 6, 5, 7, 9, 8]


@pytest.mark.parametrize("layout", [tcbf.PLANAR, tcbf.INTERLEAVED])
def test_group_per_problem_variants_equal_single_plans(layout):
    """A mix whose problems name variants of both grouped launches (and a large
    problem whose default is the ping-pong kernel): every output equals its own
    plan's bit for bit, whichever launch it ran in."""
    shapes = MIX + [(64, 1024, 512, 128)]
    variants = PP_VARIANTS + [0]
    cases = []
    for i, (b, M, N, K) in enumerate(shapes):
        shared = i == 3
        cases.append((b, M, N, K, shared) + make(140 + i, b, M, N, K, shared, layout))
    assert tcbf.Plan(64, 1024, 512, 128, tcbf.F16).info()["variant"] == 9
    log("group with per-problem variants %s, layout %d" % (variants, layout))
    tcbf.group_execute([(c[7], c[8], c[9], c[4]) for c in cases], c_layout=layout, variants=variants)
    torch.cuda.synchronize()
    for v, (b, M, N, K, shared, W, X, Wd, Xd, C) in zip(variants, cases):
        ref = single(Wd, Xd, b, M, N, K, shared, layout)
        torch.cuda.synchronize()
        got = C.cpu().numpy()
        assert not np.isnan(got).any(), (v, b, M, N, K)
        assert np.array_equal(got, ref.cpu().numpy()), (v, b, M, N, K)
    # one of the ping-pong problems against the oracle
    b, M, N, K, shared, W, X, Wd, Xd, C = cases[0]
    Ch = C.cpu().numpy().astype(np.float64)
    got = Ch[:, 0] + 1j * Ch[:, 1] if layout == tcbf.PLANAR else Ch[..., 0] + 1j * Ch[..., 1]
    Wc, Xc = wl.planar_to_complex(W), wl.planar_to_complex(X)
    check_fp_full(got, oracle.cgemm(Wc, Xc), np.matmul(np.abs(Wc), np.abs(Xc)), K)


def test_group_ping_pong_blocked_and_graph_replays():
    """Receiver-blocked weights in the grouped ping-pong launch, captured in a
    graph with a grouped 128 x 128 launch in the same call; replays equal the
    eager result."""
    shapes = MIX_BLOCKED[:6]
    variants = [9, 2, 9, 6, 9, 5]
    cases = []
    for i, (b, M, N, K) in enumerate(shapes):
        W, X, Wd, Xd, C = make(160 + i, b, M, N, K)
        cases.append((b, M, N, K, tcbf.block_weights(Wd), Xd, C, Wd))
    ws = torch.zeros(tcbf.GROUP_WORKSPACE_BYTES, dtype=torch.uint8, device="cuda:0")
    probs = [(c[4], c[5], c[6]) for c in cases]
    tcbf.group_execute(probs, workspace=ws, layout=tcbf.BLOCKED, variants=variants)
    torch.cuda.synchronize()
    for (b, M, N, K, Wb, Xd, C, Wd) in cases:
        ref = single(Wd, Xd, b, M, N, K)
        torch.cuda.synchronize()
        assert torch.equal(C, ref), (b, M, N, K)
    eager = [c[6].clone() for c in cases]
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            tcbf.group_execute(probs, workspace=ws, layout=tcbf.BLOCKED, variants=variants, stream=s)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    for r in range(3):
        for c in cases:
            c[6].fill_(float("nan"))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for c, e in zip(cases, eager):
            assert torch.equal(c[6], e), "replay %d differs" % r


def test_group_rejects_variants_a_problem_cannot_take():
    W, X, Wd, Xd, C = make(170, 1, 64, 64, 64)
    with pytest.raises(ValueError):
        tcbf.group_execute([(Wd, Xd, C)], variants=[9, 9])
    with pytest.raises(tcbf.TcbfError):
        tcbf.group_execute([(Wd, Xd, C)], variants=[1])            # the generic kernel is not grouped
    with pytest.raises(tcbf.TcbfError):
        tcbf.group_execute([(tcbf.block_weights(Wd), Xd, C)], layout=tcbf.BLOCKED, variants=[3])


def test_prepared_group_call_equals_group_execute():
    """GroupCall builds the problem table once; each call launches it again
    and gives group_execute's results bit for bit, also after the inputs
    change in place between calls."""
    cases = [make(180 + i, b, M, N, K) for i, (b, M, N, K) in enumerate(MIX[:5])]
    probs = [(c[2], c[3], c[4]) for c in cases]
    call = tcbf.GroupCall(probs)
    gen = torch.Generator(device="cuda:0")
    gen.manual_seed(9)
    for rep in range(3):
        for c in cases:
            c[4].fill_(float("nan"))
        call()
        torch.cuda.synchronize()
        got = [c[4].clone() for c in cases]
        tcbf.group_execute(probs)
        torch.cuda.synchronize()
        for g, c in zip(got, cases):
            assert not torch.isnan(g).any() and torch.equal(g, c[4]), "call %d" % rep
        for c in cases:
            c[3].copy_(torch.randint(-127, 128, c[3].shape, device="cuda:0", generator=gen).half())
