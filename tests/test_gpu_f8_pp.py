"""GPU parity of the FP8 ping-pong persistent kernel (variant 3) through the
C ABI.

Variant 3 runs 256 x 128 tiles with W as the matrix instruction's first
operand; every output takes the same products in the same order with the
same scales as in the 128 x 128 kernel (variant 1), so the two must agree bit
for bit, for per-row and per-block scales, planar and receiver-blocked codes,
planar and interleaved output, shared and strided weights, one or several
tiles per workgroup and both tile orders (a grid that is or is not a multiple
of the 8 XCDs).  Small shapes are also checked against the FP64 oracle on the
dequantised inputs (the gate of the FP8 mode, see test_gpu_f8).  Per-block
scales need every 8-stage scale group to span two stages or more
(ceil(Kp / 64) % 8 != 1); the plan must refuse the others."""
import numpy as np
import pytest

from gpu_util import log, to_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_2505_03269_amd as tcbf  # noqa: E402
from test_gpu_f8 import check_f8, dequant, host_scales, random_source  # noqa: E402

PP = 3

# (batch, M, N, K): stage counts nk = ceil(Kp / 64) in the comments
SHAPES = [
    (1, 1, 4, 1),            # nk 1: one partial tile (per-block refused)
    (2, 200, 132, 77),       # nk 2, ragged beams and samples
    (3, 257, 136, 96),       # nk 2, the last stage half a block
    (1, 300, 264, 576),      # nk 9 (per-block refused)
    (2, 256, 256, 1100),     # nk 18, a partial last scale group
    (50, 300, 264, 200),     # 300 tiles: workgroups run two tiles
    (13, 130, 260, 640),     # 39 tiles: grid not a multiple of 8; nk 10
    (1, 520, 128, 2048),     # nk 32
]


def nk_of(K):
    return (tcbf.f8_kp(K) + 63) // 64


def quantised(seed, batch, M, N, K, block, layout, nw=None):
    """Device codes and scales of random operands (quantised on the GPU)."""
    W = random_source(seed, (nw or batch, 2, M, K), "f16", 1.0)
    X = random_source(seed + 1, (batch, 2, K, N), "f16", 30.0)
    Wq, Ws = tcbf.quantize_e4m3(to_dev(W), k_major=True, block=block, out_layout=layout)
    Xq, Xs = tcbf.quantize_e4m3(to_dev(X), k_major=False, block=block, out_layout=layout)
    return Wq, Ws, Xq, Xs


def execute(plan, Wq, Xq, Ws, Xs):
    C = plan.empty_output()
    C.fill_(float("nan"))
    plan.execute(Wq, Xq, C, Ws, Xs)
    torch.cuda.synchronize()
    return C


@pytest.mark.parametrize("batch,M,N,K", SHAPES)
@pytest.mark.parametrize("dtype", [tcbf.F8_E4M3, tcbf.MXF8_E4M3])
def test_pp_equals_variant1(dtype, batch, M, N, K):
    block = 0 if dtype == tcbf.F8_E4M3 else 32
    refused = block and nk_of(K) % 8 == 1
    for layout in (tcbf.PLANAR, tcbf.BLOCKED):
        kw = dict(a_layout=layout, b_layout=layout)
        if refused:
            with pytest.raises(tcbf.TcbfError):
                tcbf.Plan(batch, M, N, K, dtype, variant=PP, **kw)
            return
        log("f8 pp dtype=%d %d x %d x %d x %d layout %d" % (dtype, batch, M, N, K, layout))
        Wq, Ws, Xq, Xs = quantised(40 + K, batch, M, N, K, block, layout)
        pp = tcbf.Plan(batch, M, N, K, dtype, variant=PP, **kw)
        assert pp.info()["tile_m"] == 256 and pp.info()["threads"] == 512
        got = execute(pp, Wq, Xq, Ws, Xs)
        ref = execute(tcbf.Plan(batch, M, N, K, dtype, variant=1, **kw), Wq, Xq, Ws, Xs)
        assert not torch.isnan(got).any()
        assert torch.equal(got, ref)
        # interleaved output
        kwc = dict(kw, c_layout=tcbf.INTERLEAVED)
        got_i = execute(tcbf.Plan(batch, M, N, K, dtype, variant=PP, **kwc), Wq, Xq, Ws, Xs)
        assert torch.equal(got_i, ref.permute(0, 2, 3, 1))
        if layout == tcbf.PLANAR and batch * M * N * K <= 2e8:
            kp = tcbf.f8_kp(K)
            Wd = dequant(Wq.cpu().numpy(), host_scales(Ws, block, kp), block, K)
            Xd = dequant(Xq.cpu().numpy(), host_scales(Xs, block, kp), block, K)
            g = got.cpu().numpy().astype(np.float64)
            check_f8(g[:, 0] + 1j * g[:, 1], Wd, Xd, K)


@pytest.mark.parametrize("dtype", [tcbf.F8_E4M3, tcbf.MXF8_E4M3])
def test_pp_shared_and_strided_weights(dtype):
    block = 0 if dtype == tcbf.F8_E4M3 else 32
    batch, M, N, K = 3, 300, 136, 640
    # one W for every batch entry
    Wq, Ws, Xq, Xs = quantised(60, batch, M, N, K, block, tcbf.BLOCKED, nw=1)
    kw = dict(a_layout=tcbf.BLOCKED, b_layout=tcbf.BLOCKED, a_shared=True)
    got = execute(tcbf.Plan(batch, M, N, K, dtype, variant=PP, **kw), Wq, Xq, Ws, Xs)
    ref = execute(tcbf.Plan(batch, M, N, K, dtype, variant=1, **kw), Wq, Xq, Ws, Xs)
    assert torch.equal(got, ref)
    # W entries a stride apart, NaN codes in the gaps
    Wq, Ws, Xq, Xs = quantised(61, batch, M, N, K, block, tcbf.PLANAR)
    per = Wq[0].numel()
    stride = per + 16 * 5
    buf = torch.full((stride * (batch - 1) + per + 64,), 0x7F, dtype=torch.uint8, device=Wq.device)
    Wst = buf.as_strided(tuple(Wq.shape), (stride,) + tuple(Wq[0].stride()))
    Wst.copy_(Wq)
    got = execute(tcbf.Plan(batch, M, N, K, dtype, variant=PP, a_batch_stride=stride), Wst, Xq, Ws, Xs)
    ref = execute(tcbf.Plan(batch, M, N, K, dtype, variant=1), Wq, Xq, Ws, Xs)
    assert not torch.isnan(got).any()
    assert torch.equal(got, ref)


@pytest.mark.parametrize("dtype", [tcbf.F8_E4M3, tcbf.MXF8_E4M3])
def test_pp_ultrasound_shape_full_output(dtype):
    """The ultrasound shape (1 x 32768 x 8192 x 256) with random codes and
    scales drawn on the device: every output of variant 3 equals variant 1's."""
    M, N, K = 32768, 256, 8192
    block = 0 if dtype == tcbf.F8_E4M3 else 32
    kw = dict(a_layout=tcbf.BLOCKED, b_layout=tcbf.BLOCKED)
    pp = tcbf.Plan(1, M, N, K, dtype, variant=PP, **kw)
    v1 = tcbf.Plan(1, M, N, K, dtype, variant=1, **kw)
    g = torch.Generator(device="cuda:0")
    g.manual_seed(5 + dtype)
    # e4m3 codes without the two NaN codes (0x7F, 0xFF)
    A = torch.randint(0, 254, pp.shape_a(), dtype=torch.uint8, device="cuda:0", generator=g)
    B = torch.randint(0, 254, pp.shape_b(), dtype=torch.uint8, device="cuda:0", generator=g)
    A = A + (A >= 0x7F).to(torch.uint8)
    B = B + (B >= 0x7F).to(torch.uint8)
    if block == 0:
        sa = torch.rand(pp.shape_a_scale(), device="cuda:0", generator=g) + 0.5
        sb = torch.rand(pp.shape_b_scale(), device="cuda:0", generator=g) + 0.5
    else:
        sa = torch.randint(120, 135, pp.shape_a_scale(), dtype=torch.uint8, device="cuda:0", generator=g)
        sb = torch.randint(120, 135, pp.shape_b_scale(), dtype=torch.uint8, device="cuda:0", generator=g)
    log("f8 pp ultrasound shape dtype=%d: execute" % dtype)
    got = execute(pp, A, B, sa, sb)
    ref = execute(v1, A, B, sa, sb)
    assert not torch.isnan(got).any()
    assert torch.equal(got, ref)


@pytest.mark.parametrize("dtype", [tcbf.F8_E4M3, tcbf.MXF8_E4M3])
def test_pp_graph_replays_match_eager(dtype):
    """The ping-pong plan captured in a HIP graph and replayed with new X
    codes quantised eagerly between replays equals variant 1 every time."""
    block = 0 if dtype == tcbf.F8_E4M3 else 32
    batch, M, N, K = 2, 520, 264, 1024
    kw = dict(a_layout=tcbf.BLOCKED, b_layout=tcbf.BLOCKED)
    Wq, Ws, Xq, Xs = quantised(80, batch, M, N, K, block, tcbf.BLOCKED)
    pp = tcbf.Plan(batch, M, N, K, dtype, variant=PP, **kw)
    v1 = tcbf.Plan(batch, M, N, K, dtype, variant=1, **kw)
    C = pp.empty_output()
    pp.execute(Wq, Xq, C, Ws, Xs)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            pp.execute(Wq, Xq, C, Ws, Xs)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    gen = torch.Generator(device="cuda:0")
    gen.manual_seed(9)
    for rep in range(3):
        X = torch.randint(-127, 128, (batch, 2, K, N), device="cuda:0", generator=gen).half()
        tcbf.quantize_e4m3(X, k_major=False, block=block, out=Xq, scales=Xs, out_layout=tcbf.BLOCKED)
        C.fill_(float("nan"))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        ref = execute(v1, Wq, Xq, Ws, Xs)
        assert torch.equal(C, ref), "replay %d" % rep


def test_pp_seeded_random_shapes():
    """Forty seeded shapes (batch 1-6, M 1-1100, N a multiple of 4 up to 700,
    K 1-3000), each dtype and code layout: variant 3 equals variant 1 bit for
    bit wherever the plan accepts it, and refuses per-block scales exactly
    where an 8-stage scale group would span one stage."""
    rng = np.random.default_rng(2025)
    for i in range(40):
        batch = int(rng.integers(1, 7))
        M = int(rng.integers(1, 1101))
        N = 4 * int(rng.integers(1, 176))
        K = int(rng.integers(1, 3001))
        dtype = tcbf.F8_E4M3 if i % 2 == 0 else tcbf.MXF8_E4M3
        layout = tcbf.PLANAR if (i // 2) % 2 == 0 else tcbf.BLOCKED
        block = 0 if dtype == tcbf.F8_E4M3 else 32
        kw = dict(a_layout=layout, b_layout=layout)
        if block and nk_of(K) % 8 == 1:
            with pytest.raises(tcbf.TcbfError):
                tcbf.Plan(batch, M, N, K, dtype, variant=PP, **kw)
            continue
        log("f8 pp random %d: dtype=%d %d x %d x %d x %d layout %d" % (i, dtype, batch, M, N, K, layout))
        Wq, Ws, Xq, Xs = quantised(500 + i, batch, M, N, K, block, layout)
        got = execute(tcbf.Plan(batch, M, N, K, dtype, variant=PP, **kw), Wq, Xq, Ws, Xs)
        ref = execute(tcbf.Plan(batch, M, N, K, dtype, variant=1, **kw), Wq, Xq, Ws, Xs)
        assert torch.equal(got, ref), "shape %d" % i
