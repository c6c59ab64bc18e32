"""GPU parity of the steering-weight generator (tcbf_steering_weights) against
the oracle's FP64 generator, through the C ABI.

Both sides evaluate the same FP64 phase with the same operations (nothing
fused); cos/sin come from different math libraries (a few FP64 ulps apart),
so a result may land on the other side of an fp16 rounding boundary: the gate
is at most 1 fp16 ulp (fp32: 1 fp32 ulp) per element, and almost all elements
must be identical.  Closed forms (whole, half and quarter turns) are exact.
"""
import numpy as np
import pytest

import oracle
import workloads as wl
from gpu_util import log, to_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_2505_03269_amd as tcbf  # noqa: E402

C0 = wl.C0


def ordered(bits16):
    """fp16 bit patterns -> integers ordered like the values (+0 and -0 both 0)."""
    b = bits16.astype(np.int32)
    return np.where(b & 0x8000, -(b & 0x7FFF), b)


def ordered32(bits32):
    b = bits32.astype(np.int64)
    return np.where(b & 0x80000000, -(b & 0x7FFFFFFF), b)


def gpu_weights(pos, dirs, freqs, dtype=torch.float16):
    W = tcbf.steering_weights(to_dev(pos), to_dev(dirs), to_dev(np.asarray(freqs, np.float64)), C0, dtype=dtype)
    torch.cuda.synchronize()
    return W.cpu().numpy()


def check_against_oracle(pos, dirs, freqs):
    ref = oracle.steering_weights(pos, dirs, freqs, C0)            # complex128 [batch, M, K]
    for dtype in (torch.float16, torch.float32):
        got = gpu_weights(pos, dirs, freqs, dtype)                  # [batch, 2, M, K]
        if dtype == torch.float16:
            rr = ref.real.astype(np.float16).view(np.uint16)
            ri = ref.imag.astype(np.float16).view(np.uint16)
            gr, gi = got[:, 0].view(np.uint16), got[:, 1].view(np.uint16)
            dr = np.abs(ordered(gr) - ordered(rr))
            di = np.abs(ordered(gi) - ordered(ri))
        else:
            rr = ref.real.astype(np.float32).view(np.uint32)
            ri = ref.imag.astype(np.float32).view(np.uint32)
            gr, gi = got[:, 0].view(np.uint32), got[:, 1].view(np.uint32)
            dr = np.abs(ordered32(gr) - ordered32(rr))
            di = np.abs(ordered32(gi) - ordered32(ri))
        n = dr.size + di.size
        exact = int((dr == 0).sum() + (di == 0).sum())
        log("steering %s: %d of %d identical, max ulp %d" % (dtype, exact, n, int(max(dr.max(), di.max()))))
        assert dr.max() <= 1 and di.max() <= 1
        assert exact >= n * 0.999


def test_random_geometry_matches_oracle():
    g = np.random.default_rng(5)
    pos = g.uniform(-1500, 1500, (300, 3))
    dirs = g.uniform(-0.2, 0.2, (70, 3))
    check_against_oracle(pos, dirs, [110e6, 150e6, 190e6])


def test_closed_forms_exact():
    pos = np.array([[0, 0, 0], [3.0, 0, 0], [2.5, 0, 0], [1.25, 0, 0]])
    dirs = np.array([[0.0, 0, 0], [1.0, 0, 0]])
    W = tcbf.steering_weights(to_dev(pos), to_dev(dirs), to_dev(np.array([1.0])), 1.0, dtype=torch.float32)
    torch.cuda.synchronize()
    w = W.cpu().numpy()[0]
    assert np.array_equal(w[0, 0], np.ones(4)) and np.array_equal(w[1, 0], np.zeros(4))  # broadside
    assert w[0, 1, 1] == 1.0 and w[1, 1, 1] == 0.0                                      # 3 whole turns
    assert w[0, 1, 2] == -1.0 and abs(w[1, 1, 2]) < 1e-15                               # half turn
    assert abs(w[0, 1, 3]) < 1e-15 and w[1, 1, 3] == 1.0                                # quarter turn


def test_c2_geometry_full_size():
    """The radio-astronomy geometry (256 channels x 1024 beams x 576
    antennas) generated on the GPU: four channels against the oracle, and all
    channels within 1 fp16 ulp of the host-generated inputs the benchmark uses."""
    ax, ay, bl, bm = wl.c2_geometry()
    pos = np.column_stack([ax, ay, np.zeros_like(ax)])
    dirs = np.column_stack([bl, bm, np.zeros_like(bl)])
    freqs = np.array([wl.c2_frequency(c) for c in range(256)])
    log("c2 steering: generate on the GPU")
    W = tcbf.steering_weights(to_dev(pos), to_dev(dirs), to_dev(freqs), C0)
    torch.cuda.synchronize()
    Wh = W.cpu().numpy()
    for c in (0, 77, 128, 255):
        ref = oracle.steering_weights(pos, dirs, freqs[c:c + 1], C0)[0]
        for p, part in ((0, ref.real), (1, ref.imag)):
            d = np.abs(ordered(Wh[c, p].view(np.uint16)) - ordered(part.astype(np.float16).view(np.uint16)))
            assert d.max() <= 1 and (d == 0).mean() >= 0.999
    geo = (ax, ay, bl, bm)
    worst = 0
    for c in range(0, 256, 15):
        host = wl.c2_weights(c, geo)
        d = np.abs(ordered(Wh[c].view(np.uint16)) - ordered(host.view(np.uint16)))
        worst = max(worst, int(d.max()))
    assert worst <= 1


def test_plane_wave_beamformed_end_to_end():
    """GPU weights -> GPU fp16 product: a plane wave arriving from beam j's
    direction adds up coherently (|B[j]| = K * |A|) in beam j."""
    g = np.random.default_rng(6)
    K, M, N, f = 192, 64, 64, 150e6
    pos = np.column_stack([g.uniform(-400, 400, (K, 2)), np.zeros(K)])
    # beams on an 8 x 8 grid of direction cosines 0.01 apart: several beam
    # widths (wavelength / aperture ~ 0.0025) between neighbours
    gl = (np.arange(8) - 3.5) * 0.01
    L, Mm = np.meshgrid(gl, gl)
    dirs = np.column_stack([L.ravel(), Mm.ravel(), np.zeros(M)])
    W = tcbf.steering_weights(to_dev(pos), to_dev(dirs), to_dev(np.array([f])), C0)
    A = 40.0 - 25.0j
    tau = pos @ dirs[:N].T / C0                        # sample n: wave from beam n's direction
    Xc = A * np.exp(-2j * np.pi * f * tau)             # [K, N]
    X = np.stack([Xc.real, Xc.imag])[None].astype(np.float16)
    plan = tcbf.Plan(1, M, N, K, tcbf.F16)
    C = plan.empty_output()
    plan.execute(W, to_dev(X), C)
    torch.cuda.synchronize()
    B = C.cpu().numpy()[0]
    Bc = B[0] + 1j * B[1]
    gain = np.abs(np.diag(Bc[:N, :N]))
    # fp16 weights and samples: each term carries ~1e-3 relative error, the sum is K terms
    assert np.allclose(gain, K * abs(A), rtol=2e-3)
    off = np.abs(Bc[:N, :N][~np.eye(N, dtype=bool)])
    assert off.max() < 0.5 * K * abs(A)     # the grid keeps other beams below ~0.18 of the main lobe


def test_e4m3_weights_from_geometry():
    """Steering weights for the FP8 mode: generated in FP64 on the GPU, rounded
    to fp32, quantised to e4m3 on the GPU (per-row scales) -- codes and scales
    bit-exact against the oracle's quantiser on the same fp32 weights -- then
    a plane wave from each beam's direction beamformed in FP8 adds up to
    K |A| in that beam (within the e4m3 rounding of both operands)."""
    g = np.random.default_rng(16)
    K, M, N, f = 192, 64, 64, 150e6
    pos = np.column_stack([g.uniform(-400, 400, (K, 2)), np.zeros(K)])
    gl = (np.arange(8) - 3.5) * 0.01
    L, Mm = np.meshgrid(gl, gl)
    dirs = np.column_stack([L.ravel(), Mm.ravel(), np.zeros(M)])
    W32 = tcbf.steering_weights(to_dev(pos), to_dev(dirs), to_dev(np.array([f])), C0, dtype=torch.float32)
    Wq, Ws = tcbf.quantize_e4m3(W32, k_major=True, block=0)
    torch.cuda.synchronize()
    w = W32.cpu().numpy()[0]
    qr, qi, sc = oracle.quantize_e4m3_rows(w[0], w[1])
    kp = tcbf.f8_kp(K)
    got = Wq.cpu().numpy()[0]
    assert np.array_equal(got[0, :, :K], qr) and np.array_equal(got[1, :, :K], qi)
    assert not got[:, :, K:].any()
    assert np.array_equal(Ws.cpu().numpy()[0].view(np.uint32), sc.view(np.uint32))
    A = 40.0 - 25.0j
    tau = pos @ dirs[:N].T / C0
    Xc = A * np.exp(-2j * np.pi * f * tau)                        # [K, N]
    X = np.stack([Xc.real, Xc.imag])[None].astype(np.float32)
    Xq, Xs = tcbf.quantize_e4m3(to_dev(X), k_major=False, block=0)
    plan = tcbf.Plan(1, M, N, kp, tcbf.F8_E4M3)
    C = plan.empty_output()
    plan.execute(Wq, Xq, C, Ws, Xs)
    torch.cuda.synchronize()
    B = C.cpu().numpy()[0]
    Bc = B[0] + 1j * B[1]
    gain = np.abs(np.diag(Bc[:N, :N]))
    assert np.allclose(gain, K * abs(A), rtol=3e-2)
    off = np.abs(Bc[:N, :N][~np.eye(N, dtype=bool)])
    assert off.max() < 0.5 * K * abs(A)


def test_rejects_bad_arguments():
    pos = torch.zeros((4, 3), dtype=torch.float64, device="cuda:0")
    dirs = torch.zeros((2, 3), dtype=torch.float64, device="cuda:0")
    fr = torch.ones(1, dtype=torch.float64, device="cuda:0")
    with pytest.raises(ValueError):
        tcbf.steering_weights(pos.float(), dirs, fr, C0)
    with pytest.raises(tcbf.TcbfError):
        tcbf.steering_weights(pos, dirs, fr, -1.0)
    with pytest.raises(ValueError):
        tcbf.steering_weights(pos, dirs, fr, C0, dtype=torch.int8)


@pytest.mark.parametrize("batch,M,K", [(2, 70, 576), (3, 33, 100), (1, 5, 7), (2, 130, 64), (1, 1, 1)])
def test_blocked_output_equals_repacked_planar(batch, M, K):
    """Weights written straight into the receiver-blocked layout are the planar
    weights repacked by tcbf_block_weights, bit for bit (zeros past K); poison
    in the output proves every element is written."""
    g = np.random.default_rng([77, batch, M, K])
    pos = np.column_stack([g.uniform(-900, 900, K), g.uniform(-900, 900, K), g.uniform(-5, 5, K)])
    dirs = np.column_stack([g.uniform(-0.05, 0.05, M), g.uniform(-0.05, 0.05, M), np.ones(M)])
    freqs = g.uniform(1.2e8, 1.8e8, batch)
    P, D, F = to_dev(pos), to_dev(dirs), to_dev(freqs)
    planar = tcbf.steering_weights(P, D, F, C0)
    out = torch.full(tcbf.blocked_shape(batch, M, K), float("nan"), dtype=torch.float16, device="cuda:0")
    blocked = tcbf.steering_weights(P, D, F, C0, out=out, out_layout=tcbf.BLOCKED)
    torch.cuda.synchronize()
    assert torch.equal(blocked.view(torch.int16), tcbf.block_weights(planar).view(torch.int16))
    with pytest.raises(ValueError):
        tcbf.steering_weights(P, D, F, C0, dtype=torch.float32, out_layout=tcbf.BLOCKED)
