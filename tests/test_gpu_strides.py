"""Descriptor fields of version 4, on the device: receiver-contiguous fp16 X
(b_k_contiguous) and W batch entries a given stride apart (a_batch_stride).

Receiver-contiguous X is checked against the FP64 oracle (relative Frobenius
and the per-element fp32 bound) and bit for bit against the same product from
X in the usual [K][N] layout on the same kernel.  Strided W is checked bit for
bit against the packed layout for every dtype and the variants that read it;
the gaps between entries hold values that would poison any output that read
them (NaN for fp16, NaN codes for FP8, flipped words for 1-bit)."""
import numpy as np
import pytest

import oracle
import workloads as wl
from gpu_util import check_fp_full, log, to_dev, words_to_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_2505_03269_amd as tcbf  # noqa: E402

KMAJOR_SHAPES = [(1, 1, 1, 1), (2, 130, 72, 100), (1, 300, 264, 576), (3, 64, 9, 33), (1, 257, 130, 8)]


def _run(plan, A, B, *scales):
    C = plan.empty_output()
    C.fill_(float("nan")) if C.dtype == torch.float32 else C.fill_(-7)
    plan.execute(A, B, C, *scales)
    torch.cuda.synchronize()
    return C


@pytest.mark.parametrize("batch,M,N,K", KMAJOR_SHAPES)
@pytest.mark.parametrize("b_layout", [tcbf.PLANAR, tcbf.INTERLEAVED])
def test_receiver_contiguous_x(batch, M, N, K, b_layout):
    W, X = wl.random_f16_case(700 + K, batch, M, N, K)
    log("receiver-contiguous X: %d x %d x %d x %d, layout %d" % (batch, M, N, K, b_layout))
    Wd = to_dev(W)
    if b_layout == tcbf.PLANAR:
        Xk = np.ascontiguousarray(X.transpose(0, 1, 3, 2))     # [batch, 2, N, K]
        Xs = X                                                 # [batch, 2, K, N]
    else:
        Xk = np.ascontiguousarray(X.transpose(0, 3, 2, 1))     # [batch, N, K, 2]
        Xs = np.ascontiguousarray(X.transpose(0, 2, 3, 1))     # [batch, K, N, 2]
    plan = tcbf.Plan(batch, M, N, K, tcbf.F16, b_layout=b_layout, b_k_contiguous=True)
    assert plan.info()["variant"] == 1 and plan.shape_b() == Xk.shape
    got = _run(plan, Wd, to_dev(Xk))
    ref_plan = tcbf.Plan(batch, M, N, K, tcbf.F16, b_layout=b_layout, variant=1)
    ref = _run(ref_plan, Wd, to_dev(Xs))
    assert torch.equal(got, ref)
    g = got.cpu().numpy().astype(np.float64)
    Wc, Xc = wl.planar_to_complex(W), wl.planar_to_complex(X)
    check_fp_full(g[:, 0] + 1j * g[:, 1], oracle.cgemm(Wc, Xc), np.matmul(np.abs(Wc), np.abs(Xc)), K)


def _strided(t, stride, fill):
    """A copy of contiguous t [batch, ...] whose batch entries sit `stride`
    elements apart in a buffer filled with `fill` elsewhere."""
    batch = t.shape[0]
    per = t[0].numel()
    buf = torch.full((stride * (batch - 1) + per + 64,), fill, dtype=t.dtype, device=t.device)
    inner = t[0].stride()
    v = buf.as_strided(tuple(t.shape), (stride,) + tuple(inner))
    v.copy_(t)
    return v


@pytest.mark.parametrize("a_layout,variant", [(tcbf.PLANAR, 1), (tcbf.PLANAR, 2), (tcbf.PLANAR, 6), (tcbf.PLANAR, 8),
                                              (tcbf.PLANAR, 9), (tcbf.BLOCKED, 2), (tcbf.BLOCKED, 9),
                                              (tcbf.INTERLEAVED, 1)])
def test_strided_fp16_weights(a_layout, variant):
    batch, M, N, K = 3, 300, 264, 200
    W, X = wl.random_f16_case(810 + variant, batch, M, N, K)
    Wd = to_dev(W)
    if a_layout == tcbf.BLOCKED:
        Wd = tcbf.block_weights(Wd)
    elif a_layout == tcbf.INTERLEAVED:
        Wd = Wd.permute(0, 2, 3, 1).contiguous()
    Xd = to_dev(X)
    per = Wd[0].numel()
    stride = per + 8 * 37
    Ws = _strided(Wd, stride, float("nan"))
    log("strided fp16 W: layout %d variant %d stride %d (entry %d)" % (a_layout, variant, stride, per))
    plan = tcbf.Plan(batch, M, N, K, tcbf.F16, a_layout=a_layout, variant=variant, a_batch_stride=stride)
    dense = tcbf.Plan(batch, M, N, K, tcbf.F16, a_layout=a_layout, variant=variant)
    got, ref = _run(plan, Ws, Xd), _run(dense, Wd, Xd)
    assert not torch.isnan(got).any()
    assert torch.equal(got, ref)


@pytest.mark.parametrize("dtype,layout", [(tcbf.F8_E4M3, tcbf.PLANAR), (tcbf.F8_E4M3, tcbf.BLOCKED),
                                          (tcbf.MXF8_E4M3, tcbf.PLANAR), (tcbf.MXF8_E4M3, tcbf.BLOCKED)])
def test_strided_fp8_codes(dtype, layout):
    batch, M, N, K = 2, 200, 136, 300
    block = 32 if dtype == tcbf.MXF8_E4M3 else 0
    W, X = wl.random_f16_case(830 + dtype, batch, M, N, K)
    Wq, Ws = tcbf.quantize_e4m3(to_dev(W), k_major=True, block=block, out_layout=layout)
    Xq, Xs = tcbf.quantize_e4m3(to_dev(X), k_major=False, block=block, out_layout=layout)
    per = Wq[0].numel()
    stride = per + 16 * 9
    Wqs = _strided(Wq, stride, 0x7F)   # e4m3 NaN codes in the gaps
    log("strided FP8 codes: dtype %d layout %d stride %d (entry %d)" % (dtype, layout, stride, per))
    plan = tcbf.Plan(batch, M, N, K, dtype, a_layout=layout, b_layout=layout, a_batch_stride=stride)
    dense = tcbf.Plan(batch, M, N, K, dtype, a_layout=layout, b_layout=layout)
    got, ref = _run(plan, Wqs, Xq, Ws, Xs), _run(dense, Wq, Xq, Ws, Xs)
    assert not torch.isnan(got).any()
    assert torch.equal(got, ref)


@pytest.mark.parametrize("variant", [1, 2, 3])
def test_strided_packed_weights(variant):
    batch, M, N, K = 3, 140, 72, 1024
    Wp, Xp = wl.random_bits_case(850 + variant, batch, M, N, K)
    Wd, Xd = words_to_dev(Wp), words_to_dev(Xp)
    per = Wd[0].numel()
    stride = per + 4 * 11
    Wds = _strided(Wd, stride, -1)
    log("strided packed W: variant %d stride %d (entry %d)" % (variant, stride, per))
    plan = tcbf.Plan(batch, M, N, K, tcbf.INT1, variant=variant, a_batch_stride=stride)
    dense = tcbf.Plan(batch, M, N, K, tcbf.INT1, variant=variant)
    got, ref = _run(plan, Wds, Xd), _run(dense, Wd, Xd)
    assert torch.equal(got, ref)
    # and the dense result against the popcount oracle
    cont = np.ascontiguousarray
    rr, ri = oracle.cgemm_1bit_popc(cont(Wp[:, 0]), cont(Wp[:, 1]), cont(Xp[:, 0]), cont(Xp[:, 1]), K)
    g = ref.cpu().numpy().astype(np.int64)
    assert np.array_equal(g[:, 0], rr) and np.array_equal(g[:, 1], ri)


def test_binding_checks_the_stride_of_the_view():
    batch, M, N, K = 2, 64, 64, 64
    W, X = wl.random_f16_case(870, batch, M, N, K)
    Wd, Xd = to_dev(W), to_dev(X)
    stride = Wd[0].numel() + 64
    plan = tcbf.Plan(batch, M, N, K, tcbf.F16, a_batch_stride=stride)
    with pytest.raises(ValueError):
        plan.execute(Wd, Xd, plan.empty_output())        # packed W given to a strided plan
    with pytest.raises(ValueError):
        plan.execute(_strided(Wd, stride + 8, 0.0), Xd, plan.empty_output())
