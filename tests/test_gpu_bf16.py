"""GPU parity of the bfloat16 mode (TCBF_BF16) against the FP64 oracle.

Inputs are rounded to bfloat16 on the host side of the test (torch's
round-to-nearest-even cast); the oracle takes the rounded values exactly
(every bfloat16 is a float32), so the gate is the fp16 mode's: relative
Frobenius error <= 2e-3 per channel and the per-element fp32 summation bound
(the product of two bfloat16 values is exact in fp32).  Variants 1, 2 and 9
must agree bit for bit, and blocked weights with planar ones."""
import numpy as np
import pytest

import oracle
import workloads as wl
from gpu_util import check_fp_entries, check_fp_full, log

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_2505_03269_amd as tcbf  # noqa: E402


def bf16_case(seed, batch, M, N, K):
    """Device bfloat16 W [batch, 2, M, K], X [batch, 2, K, N] and their exact
    float64 values."""
    W, X = wl.random_f16_case(seed, batch, M, N, K)
    Wb = torch.from_numpy(W.astype(np.float32)).to(torch.bfloat16)
    Xb = torch.from_numpy(X.astype(np.float32) * 3.0).to(torch.bfloat16)
    return Wb.to("cuda:0"), Xb.to("cuda:0"), Wb.float().numpy().astype(np.float64), Xb.float().numpy().astype(np.float64)


def run(plan, A, B):
    C = plan.empty_output()
    C.fill_(float("nan"))
    plan.execute(A, B, C)
    torch.cuda.synchronize()
    return C


SHAPES = [(1, 1, 1, 1), (2, 130, 72, 100), (1, 300, 264, 576), (3, 257, 136, 64), (2, 1024, 512, 96)]


@pytest.mark.parametrize("batch,M,N,K", SHAPES)
def test_bf16_matches_oracle_and_variants_agree(batch, M, N, K):
    A, B, W, X = bf16_case(900 + K, batch, M, N, K)
    plan = tcbf.Plan(batch, M, N, K, tcbf.BF16)
    log("bf16 %d x %d x %d x %d: default variant %d" % (batch, M, N, K, plan.info()["variant"]))
    C = run(plan, A, B)
    g = C.cpu().numpy().astype(np.float64)
    Wc, Xc = W[:, 0] + 1j * W[:, 1], X[:, 0] + 1j * X[:, 1]
    check_fp_full(g[:, 0] + 1j * g[:, 1], oracle.cgemm(Wc, Xc), np.matmul(np.abs(Wc), np.abs(Xc)), K)
    for v in (1, 2, 9):
        try:
            pv = tcbf.Plan(batch, M, N, K, tcbf.BF16, variant=v)
        except tcbf.TcbfError:
            continue
        assert torch.equal(run(pv, A, B), C), "variant %d" % v


def test_bf16_blocked_weights_and_layouts():
    batch, M, N, K = 2, 300, 264, 200
    A, B, W, X = bf16_case(950, batch, M, N, K)
    ref = run(tcbf.Plan(batch, M, N, K, tcbf.BF16, variant=1), A, B)
    Ab = tcbf.block_weights(A)
    assert Ab.dtype == torch.bfloat16
    for v in (2, 9):
        p = tcbf.Plan(batch, M, N, K, tcbf.BF16, a_layout=tcbf.BLOCKED, variant=v)
        assert torch.equal(run(p, Ab, B), ref), "blocked, variant %d" % v
    # interleaved W, X and output on the generic kernel, receiver-contiguous X
    Ai = A.permute(0, 2, 3, 1).contiguous()
    Bi = B.permute(0, 2, 3, 1).contiguous()
    p = tcbf.Plan(batch, M, N, K, tcbf.BF16, a_layout=tcbf.INTERLEAVED, b_layout=tcbf.INTERLEAVED,
                  c_layout=tcbf.INTERLEAVED)
    assert p.info()["variant"] == 1
    got = run(p, Ai, Bi)
    assert torch.equal(got.permute(0, 3, 1, 2), ref)
    pk = tcbf.Plan(batch, M, N, K, tcbf.BF16, b_k_contiguous=True)
    assert torch.equal(run(pk, A, B.transpose(2, 3).contiguous()), ref)


def test_bf16_radio_astronomy_shape_sampled():
    """The radio-astronomy shape (256 x 1024 x 576 x 4096) in bfloat16 on the
    ping-pong kernel, 8000 sampled entries of 12 channels plus tile corners
    against the oracle."""
    cfg = wl.WORKLOADS["radio-astro-fp16"]
    batch, M, N, K = cfg["batch"], cfg["M"], cfg["N"], cfg["K"]
    g = torch.Generator(device="cuda:0")
    g.manual_seed(77)
    A = torch.randn((batch, 2, M, K), device="cuda:0", generator=g).to(torch.bfloat16)
    B = torch.randint(-127, 128, (batch, 2, K, N), device="cuda:0", generator=g).to(torch.bfloat16)
    plan = tcbf.Plan(batch, M, N, K, tcbf.BF16, a_layout=tcbf.BLOCKED)
    assert plan.info()["variant"] == 9
    log("bf16 c2 shape: execute")
    C = run(plan, tcbf.block_weights(A), B)
    rng = np.random.default_rng(5)
    chans = rng.choice(batch, 12, replace=False)
    cs, ms, ns = chans[rng.integers(0, 12, 8000)], rng.integers(0, M, 8000), rng.integers(0, N, 8000)
    corner = np.array([0, 255, 256, M - 1])
    cs = np.concatenate([cs, np.zeros(16, int)])
    ms = np.concatenate([ms, np.repeat(corner, 4)])
    ns = np.concatenate([ns, np.tile([0, 127, 128, N - 1], 4)])
    got = np.empty(cs.size, complex)
    ref = np.empty(cs.size, complex)
    absdot = np.empty(cs.size)
    Ch = C[torch.from_numpy(cs).cuda(), :, torch.from_numpy(ms).cuda(), torch.from_numpy(ns).cuda()].cpu().numpy()
    got[:] = Ch[:, 0] + 1j * Ch[:, 1]
    for c in np.unique(cs):
        sel = np.nonzero(cs == c)[0]
        Wc = A[c].float().cpu().numpy().astype(np.float64)
        Xc = B[c].float().cpu().numpy().astype(np.float64)
        Wz = (Wc[0] + 1j * Wc[1])[None]
        Xz = (Xc[0] + 1j * Xc[1])[None]
        z = np.zeros(sel.size, np.int64)
        ref[sel] = oracle.cgemm_entries(Wz, Xz, z, ms[sel], ns[sel])
        absdot[sel] = oracle.abs_dot_entries(Wz, Xz, z, ms[sel], ns[sel])
    check_fp_entries(got, ref, absdot, K)
    log("bf16 c2 sampled rel Frobenius %.3e" % (np.linalg.norm(got - ref) / np.linalg.norm(ref)))
