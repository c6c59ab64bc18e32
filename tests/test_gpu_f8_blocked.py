"""GPU checks of the receiver-blocked FP8 operand layout (TCBF_BLOCKED).

The quantiser's blocked output is its planar output rearranged into blocks
of 64 receivers (a data movement: the codes must be identical, with zero
codes past Kp), and its scales do not depend on the output layout.  Products
of blocked operands must be bitwise identical to those of planar operands
(the kernel feeds the matrix unit the same fragments in the same order), so
the dequantised-oracle gate of the planar FP8 tests carries over; it is
checked directly here as well."""
import numpy as np
import pytest

import workloads as wl
from gpu_util import c_inter_to_complex, c_planar_to_complex, log, to_dev
from test_gpu_f8 import check_f8, dequant, host_scales, random_source, src_shape

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_2505_03269_amd as tcbf  # noqa: E402


def reblock(codes):
    """Planar codes [b, 2, rows, Kp] -> [b, 2, ceil(Kp/64), rows, 64], zero past Kp."""
    b, _, rows, kp = codes.shape
    kb = (kp + 63) // 64
    pad = np.zeros((b, 2, rows, kb * 64), codes.dtype)
    pad[..., :kp] = codes
    return np.ascontiguousarray(pad.reshape(b, 2, rows, kb, 64).transpose(0, 1, 3, 2, 4))


@pytest.mark.parametrize("block", [0, 32])
@pytest.mark.parametrize("k_major", [True, False])
@pytest.mark.parametrize("layout", [tcbf.PLANAR, tcbf.INTERLEAVED])
@pytest.mark.parametrize("K", [1, 40, 64, 72, 200, 576])
def test_quantiser_blocked_output(K, layout, k_major, block):
    """Blocked codes = planar codes rearranged (poison in the output proves
    every byte, padding included, is written); scales bit-identical."""
    batch, rows = 2, 70
    log("f8 quantise blocked: K=%d layout=%d k_major=%d block=%d" % (K, layout, k_major, block))
    src = to_dev(random_source(40 + K, src_shape(batch, rows, K, k_major, layout), "f16"))
    pc, ps = tcbf.quantize_e4m3(src, k_major=k_major, layout=layout, block=block)
    shape = tcbf.f8_codes_shape(batch, rows, K, tcbf.BLOCKED)
    out = torch.full(shape, 0xA5, dtype=torch.uint8, device="cuda:0")
    bc, bs = tcbf.quantize_e4m3(src, k_major=k_major, layout=layout, block=block, out=out,
                                out_layout=tcbf.BLOCKED)
    torch.cuda.synchronize()
    assert np.array_equal(bc.cpu().numpy(), reblock(pc.cpu().numpy()))
    if block == 0:
        assert torch.equal(ps.view(torch.int32), bs.view(torch.int32))
    else:
        a = tcbf.mx_scales_to_rows(ps.cpu().numpy(), K)  # written codes only (the rest is padding)
        b = tcbf.mx_scales_to_rows(bs.cpu().numpy(), K)
        assert np.array_equal(a, b)


def quantised_pair(seed, batch, M, N, K, block, shared=False):
    nw = 1 if shared else batch
    W = to_dev(random_source(seed, (nw, 2, M, K), "f16", 1.0))
    X = to_dev(random_source(seed + 1, (batch, 2, K, N), "f16", 30.0))
    planar = (tcbf.quantize_e4m3(W, k_major=True, block=block), tcbf.quantize_e4m3(X, k_major=False, block=block))
    blocked = (tcbf.quantize_e4m3(W, k_major=True, block=block, out_layout=tcbf.BLOCKED),
               tcbf.quantize_e4m3(X, k_major=False, block=block, out_layout=tcbf.BLOCKED))
    return planar, blocked


def run(pair, batch, M, N, K, dtype, layout, c_layout=tcbf.PLANAR, shared=False, variant=0):
    (Wq, Ws), (Xq, Xs) = pair
    plan = tcbf.Plan(batch, M, N, K, dtype, a_layout=layout, b_layout=layout, c_layout=c_layout,
                     a_shared=shared, variant=variant)
    C = plan.empty_output()
    plan.execute(Wq, Xq, C, Ws, Xs)
    torch.cuda.synchronize()
    Ch = C.cpu().numpy()
    return c_planar_to_complex(Ch) if c_layout == tcbf.PLANAR else c_inter_to_complex(Ch)


SHAPES = [(2, 160, 136, 300), (1, 128, 128, 64), (3, 70, 36, 40), (1, 257, 260, 576), (2, 64, 64, 100),
          (1, 1, 4, 1), (1, 300, 128, 1000)]


@pytest.mark.parametrize("batch,M,N,K", SHAPES)
@pytest.mark.parametrize("dtype", [tcbf.F8_E4M3, tcbf.MXF8_E4M3])
def test_blocked_products_match_planar(dtype, batch, M, N, K):
    """Ragged rows, Kp % 64 == 32 tails (the last block half past Kp), both
    ring depths, both output layouts; and the oracle gate on the dequantised
    inputs."""
    block = 0 if dtype == tcbf.F8_E4M3 else 32
    log("f8 blocked product: dtype=%d batch=%d M=%d N=%d K=%d" % (dtype, batch, M, N, K))
    planar, blocked = quantised_pair(50, batch, M, N, K, block)
    base = run(planar, batch, M, N, K, dtype, tcbf.PLANAR)
    for v in (0, 1, 2):
        got = run(blocked, batch, M, N, K, dtype, tcbf.BLOCKED, variant=v)
        assert np.array_equal(got, base), "variant %d differs from the planar product" % v
    got_il = run(blocked, batch, M, N, K, dtype, tcbf.BLOCKED, c_layout=tcbf.INTERLEAVED)
    assert np.array_equal(got_il, base)
    kp = tcbf.f8_kp(K)
    (Wq, Ws), (Xq, Xs) = planar
    Wd = dequant(Wq.cpu().numpy(), host_scales(Ws, block, kp), block, K)
    Xd = dequant(Xq.cpu().numpy(), host_scales(Xs, block, kp), block, K)
    check_f8(got, Wd, Xd, K)


@pytest.mark.parametrize("dtype", [tcbf.F8_E4M3, tcbf.MXF8_E4M3])
def test_blocked_shared_weights(dtype):
    block = 0 if dtype == tcbf.F8_E4M3 else 32
    batch, M, N, K = 3, 130, 64, 200
    planar, blocked = quantised_pair(60, batch, M, N, K, block, shared=True)
    base = run(planar, batch, M, N, K, dtype, tcbf.PLANAR, shared=True)
    got = run(blocked, batch, M, N, K, dtype, tcbf.BLOCKED, shared=True)
    assert np.array_equal(got, base)


def test_mixed_layouts_rejected():
    with pytest.raises(tcbf.TcbfError):
        tcbf.Plan(1, 64, 64, 64, tcbf.F8_E4M3, a_layout=tcbf.BLOCKED)
    with pytest.raises(tcbf.TcbfError):
        tcbf.Plan(1, 64, 64, 64, tcbf.MXF8_E4M3, b_layout=tcbf.BLOCKED)
    plan = tcbf.Plan(1, 64, 64, 100, tcbf.F8_E4M3, a_layout=tcbf.BLOCKED, b_layout=tcbf.BLOCKED)
    assert plan.shape_a() == (1, 2, 2, 64, 64) and plan.shape_b() == (1, 2, 2, 64, 64)
    with pytest.raises(ValueError):   # planar codes handed to a blocked plan
        plan.execute(torch.zeros((1, 2, 64, 128), dtype=torch.uint8, device="cuda:0"),
                     torch.zeros((1, 2, 2, 64, 64), dtype=torch.uint8, device="cuda:0"), plan.empty_output(),
                     torch.ones((1, 64), device="cuda:0"), torch.ones((1, 64), device="cuda:0"))


@pytest.mark.parametrize("dtype", [tcbf.F8_E4M3, tcbf.MXF8_E4M3])
def test_c4_full_size_blocked_equals_planar(dtype):
    """The ultrasound workload (1 x 32768 x 8192 x 256) in the launch configuration the
    benchmark times: the whole output equals the planar product bit for bit."""
    block = 0 if dtype == tcbf.F8_E4M3 else 32
    cfg = wl.WORKLOADS["ultrasound-fp16"]
    log("c4 f8 blocked: dtype=%d" % dtype)
    W, X = wl.c4_channel(0)
    A, B = to_dev(W[None]), to_dev(X[None])
    del W, X
    M, N, K = cfg["M"], cfg["N"], cfg["K"]
    pw, px = tcbf.quantize_e4m3(A, k_major=True, block=block), tcbf.quantize_e4m3(B, k_major=False, block=block)
    bw = tcbf.quantize_e4m3(A, k_major=True, block=block, out_layout=tcbf.BLOCKED)
    bx = tcbf.quantize_e4m3(B, k_major=False, block=block, out_layout=tcbf.BLOCKED)
    del A, B
    pp = tcbf.Plan(1, M, N, K, dtype)
    pb = tcbf.Plan(1, M, N, K, dtype, a_layout=tcbf.BLOCKED, b_layout=tcbf.BLOCKED)
    Cp, Cb = pp.empty_output(), pb.empty_output()
    pp.execute(pw[0], px[0], Cp, pw[1], px[1])
    pb.execute(bw[0], bx[0], Cb, bw[1], bx[1])
    torch.cuda.synchronize()
    assert torch.equal(Cp, Cb)
