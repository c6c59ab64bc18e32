"""GPU checks of the receiver-blocked weight layout (TCBF_BLOCKED).

The repack (tcbf_block_weights) is a pure data movement: every bit pattern is
copied to its place and receivers past K become +0.  Products with blocked
weights must be bitwise identical to those with planar weights (the kernel
feeds the matrix unit the same fragments in the same order; only the
addresses the W tiles are fetched from differ), and so within the oracle
gate, which is checked directly as well."""
import numpy as np
import pytest

import oracle
import workloads as wl
from gpu_util import c_inter_to_complex, c_planar_to_complex, check_fp_full, log, to_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_2505_03269_amd as tcbf  # noqa: E402


def blocked_expected(bits):
    """Planar [nb, 2, M, K] 16-bit words -> [nb, 2, ceil(K/32), M, 32], zero past K."""
    nb, _, M, K = bits.shape
    kb = (K + 31) // 32
    pad = np.zeros((nb, 2, M, kb * 32), bits.dtype)
    pad[..., :K] = bits
    return np.ascontiguousarray(pad.reshape(nb, 2, M, kb, 32).transpose(0, 1, 3, 2, 4))


@pytest.mark.parametrize("nb,M,K,layout", [
    (1, 1, 1, tcbf.PLANAR), (2, 100, 100, tcbf.PLANAR), (3, 64, 576, tcbf.PLANAR), (1, 257, 40, tcbf.PLANAR),
    (1, 33, 37, tcbf.INTERLEAVED), (2, 128, 64, tcbf.INTERLEAVED), (1, 5, 4, tcbf.INTERLEAVED),
    (2, 70, 30, tcbf.INTERLEAVED),
])
def test_block_weights_exact(nb, M, K, layout):
    """Random 16-bit patterns (NaN and infinity encodings included) land bit
    for bit; the padding is +0; poison in the output proves every element is
    written."""
    log("block_weights: nb=%d M=%d K=%d layout=%d" % (nb, M, K, layout))
    g = np.random.default_rng([31, nb, M, K, layout])
    bits = g.integers(0, 1 << 16, size=(nb, 2, M, K), dtype=np.uint16)
    src = bits if layout == tcbf.PLANAR else np.ascontiguousarray(bits.transpose(0, 2, 3, 1))
    S = to_dev(src.view(np.float16))
    out = torch.full(tcbf.blocked_shape(nb, M, K), float("nan"), dtype=torch.float16, device="cuda:0")
    tcbf.block_weights(S, layout, out=out)
    torch.cuda.synchronize()
    got = out.cpu().numpy().view(np.uint16)
    assert np.array_equal(got, blocked_expected(bits))


def _run(A, X, M, K, a_layout, c_layout=tcbf.PLANAR, shared=False, variant=0):
    batch, N = X.shape[0], X.shape[3]
    plan = tcbf.Plan(batch, M, N, K, tcbf.F16, a_layout=a_layout, c_layout=c_layout, a_shared=shared,
                     variant=variant)
    C = plan.empty_output()
    plan.execute(A, to_dev(X) if isinstance(X, np.ndarray) else X, C)
    torch.cuda.synchronize()
    Ch = C.cpu().numpy()
    return (c_planar_to_complex(Ch) if c_layout == tcbf.PLANAR else c_inter_to_complex(Ch)), plan


BLOCKED_SHAPES = [(2, 200, 136, 100), (3, 256, 256, 576), (1, 130, 8, 7), (2, 64, 64, 33), (1, 257, 392, 576),
                  (1, 1, 8, 1), (2, 129, 264, 520), (1, 1024, 512, 4096)]


@pytest.mark.parametrize("batch,M,N,K", BLOCKED_SHAPES)
def test_blocked_products_match_planar(batch, M, N, K):
    """Ragged beams and samples, receiver counts that are not multiples of 8
    or 32 (the last block's padding meets X rows read as zero), every variant
    that reads blocked weights, both output layouts."""
    log("blocked product: batch=%d M=%d N=%d K=%d" % (batch, M, N, K))
    W, X = wl.random_f16_case(17, batch, M, N, K)
    planar, _ = _run(to_dev(W), X, M, K, tcbf.PLANAR)
    Wc, Xc = wl.planar_to_complex(W), wl.planar_to_complex(X)
    check_fp_full(planar, oracle.cgemm(Wc, Xc), np.matmul(np.abs(Wc), np.abs(Xc)), K)
    Wb = tcbf.block_weights(to_dev(W))
    Xd = to_dev(X)
    names = {8: "cgemm_f16_split_kernel", 9: "cgemm_f16_pp_kernel"}
    for v in (0, 2, 5, 6, 8, 9):
        got, plan = _run(Wb, Xd, M, K, tcbf.BLOCKED, variant=v)
        assert plan.info()["kernel_name"] == names.get(v, "cgemm_f16_fast_kernel")
        assert np.array_equal(got, planar), "blocked weights, variant %d, differ from planar" % v
        if v == 9:
            got_il, _ = _run(Wb, Xd, M, K, tcbf.BLOCKED, c_layout=tcbf.INTERLEAVED, variant=v)
            assert np.array_equal(got_il, planar), "blocked weights, variant 9, interleaved output differs"
    got_il, _ = _run(Wb, Xd, M, K, tcbf.BLOCKED, c_layout=tcbf.INTERLEAVED)
    assert np.array_equal(got_il, planar)


def test_blocked_shared_weights():
    batch, M, N, K = 4, 130, 64, 72
    W, X = wl.random_f16_case(19, batch, M, N, K, shared_w=True)
    planar, _ = _run(to_dev(W), X, M, K, tcbf.PLANAR, shared=True)
    Wb = tcbf.block_weights(to_dev(W))
    assert tuple(Wb.shape) == tcbf.blocked_shape(1, M, K)
    got, _ = _run(Wb, X, M, K, tcbf.BLOCKED, shared=True)
    assert np.array_equal(got, planar)


def test_blocked_from_interleaved_weights():
    batch, M, N, K = 2, 96, 128, 200
    W, X = wl.random_f16_case(23, batch, M, N, K)
    Wi = to_dev(np.ascontiguousarray(W.transpose(0, 2, 3, 1)))
    Wb = tcbf.block_weights(Wi, tcbf.INTERLEAVED)
    assert torch.equal(Wb, tcbf.block_weights(to_dev(W)))
    planar, _ = _run(to_dev(W), X, M, K, tcbf.PLANAR)
    got, _ = _run(Wb, X, M, K, tcbf.BLOCKED)
    assert np.array_equal(got, planar)


def test_blocked_rejects_bad_tensors():
    plan = tcbf.Plan(1, 64, 64, 40, tcbf.F16, a_layout=tcbf.BLOCKED)
    assert plan.shape_a() == tcbf.blocked_shape(1, 64, 40)
    B = torch.zeros(plan.shape_b(), dtype=torch.float16, device="cuda:0")
    C = plan.empty_output()
    with pytest.raises(ValueError):
        plan.execute(torch.zeros((1, 2, 64, 40), dtype=torch.float16, device="cuda:0"), B, C)
    with pytest.raises(ValueError):
        tcbf.block_weights(torch.zeros((1, 2, 8, 8), dtype=torch.float32, device="cuda:0"))
    with pytest.raises(ValueError):
        tcbf.block_weights(torch.zeros((1, 2, 8, 8), dtype=torch.float16, device="cuda:0"), layout=tcbf.BLOCKED)


def test_c2_full_size_blocked_equals_planar():
    """The radio-astronomy workload at its full size in the launch configuration the benchmark
    times (blocked weights, default variant): the whole output equals the
    planar-weight product bit for bit (that product is checked against the
    oracle on sampled entries by the fp16 tests)."""
    cfg = wl.WORKLOADS["radio-astro-fp16"]
    log("c2 blocked: generating inputs")
    W, X = wl.generate_c2()
    A, B = to_dev(W), to_dev(X)
    del W, X
    pp = tcbf.Plan(cfg["batch"], cfg["M"], cfg["N"], cfg["K"], tcbf.F16)
    pb = tcbf.Plan(cfg["batch"], cfg["M"], cfg["N"], cfg["K"], tcbf.F16, a_layout=tcbf.BLOCKED)
    assert pb.info()["variant"] == pp.info()["variant"] == 9
    Ab = tcbf.block_weights(A)
    Cp, Cb = pp.empty_output(), pb.empty_output()
    log("c2 blocked: execute both")
    pp.execute(A, B, Cp)
    pb.execute(Ab, B, Cb)
    torch.cuda.synchronize()
    assert torch.equal(Cp, Cb)
