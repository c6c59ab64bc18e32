"""Allocation-free grouped launch (tcbf_group_execute_noalloc).

The entry point runs the grouped launch of tcbf_group_execute with its tile
counter in the library's per-GPU scratch array instead of a caller workspace.
Its outputs must equal tcbf_group_execute's bit for bit (same kernels, same
tile order), on two calls in a row, the second one smaller than the first (the
counter must be reset by every call, whatever the previous call left in it).
"""
import numpy as np
import pytest

import workloads as wl
from gpu_util import log, to_dev, words_to_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_2505_03269_amd as tcbf  # noqa: E402

BIG = [(1, 300, 264, 576), (2, 128, 128, 64), (3, 200, 392, 200), (1, 64, 1024, 2048), (2, 513, 136, 96)]
SMALL = [(1, 96, 64, 40), (1, 40, 24, 16)]


def f16_problems(seed, shapes, layout):
    probs = []
    for i, (b, M, N, K) in enumerate(shapes):
        W, X = wl.random_f16_case(seed + i, b, M, N, K)
        Cshape = (b, 2, M, N) if layout == tcbf.PLANAR else (b, M, N, 2)
        probs.append((to_dev(W), to_dev(X), torch.full(Cshape, float("nan"), device="cuda:0")))
    return probs


def int1_problems(seed, shapes):
    probs = []
    for i, (b, M, N, K) in enumerate(shapes):
        Wp, Xp = wl.random_bits_case(seed + i, b, M, N, K)
        probs.append((words_to_dev(Wp), words_to_dev(Xp),
                      torch.full((b, 2, M, N), -7, dtype=torch.int32, device="cuda:0"), K))
    return probs


def f8_problems(seed, shapes):
    probs = []
    for i, (b, M, N, K) in enumerate(shapes):
        W, X = wl.random_f16_case(seed + i, b, M, N, K)
        Wq, Ws = tcbf.quantize_e4m3(to_dev(W), k_major=True, block=0)
        Xq, Xs = tcbf.quantize_e4m3(to_dev(X), k_major=False, block=0)
        probs.append((Wq, Xq, torch.full((b, 2, M, N), float("nan"), device="cuda:0"), Ws, Xs))
    return probs


def with_fresh_outputs(probs):
    """The same problems with outputs of their own (filled with a marker)."""
    out = []
    for p in probs:
        C = p[2].clone().fill_(-7 if p[2].dtype == torch.int32 else float("nan"))
        out.append(tuple(p[:2]) + (C,) + tuple(p[3:]))
    return out


def check_pair(make, dtype, layout=tcbf.PLANAR):
    for call, shapes in enumerate((BIG, SMALL)):
        probs = make(shapes)
        ref = with_fresh_outputs(probs)
        log("noalloc dtype %d layout %d call %d: %d problems" % (dtype, layout, call, len(probs)))
        tcbf.group_execute_noalloc(probs, c_layout=layout, dtype=dtype)
        tcbf.group_execute(ref, c_layout=layout, dtype=dtype)
        torch.cuda.synchronize()
        for p, r in zip(probs, ref):
            got, want = p[2].cpu().numpy(), r[2].cpu().numpy()
            if got.dtype == np.float32:
                assert not np.isnan(want).any()
            assert np.array_equal(got, want), (dtype, layout, call, tuple(p[2].shape))


@pytest.mark.parametrize("layout", [tcbf.PLANAR, tcbf.INTERLEAVED])
def test_noalloc_f16_equals_workspace_launch(layout):
    check_pair(lambda shapes: f16_problems(500, shapes, layout), tcbf.F16, layout)


def test_noalloc_int1_equals_workspace_launch():
    check_pair(lambda shapes: int1_problems(520, shapes), tcbf.INT1)


def test_noalloc_f8_equals_workspace_launch():
    check_pair(lambda shapes: f8_problems(540, shapes), tcbf.F8_E4M3)


def test_noalloc_rejects_bad_arguments():
    probs = f16_problems(560, [(1, 64, 64, 64)], tcbf.PLANAR)
    with pytest.raises(ValueError):
        tcbf.group_execute_noalloc(probs * (tcbf.GROUP_MAX + 1))
    arr = tcbf._group_table(probs, tcbf.PLANAR, tcbf.F16, tcbf.PLANAR)
    L = tcbf.lib()
    assert L.tcbf_group_execute_noalloc(0, tcbf.F16, 5, arr, 1, None) == 1            # unknown output layout
    assert L.tcbf_group_execute_noalloc(0, tcbf.F16, 0, arr, 0, None) == 1            # no problems
    assert L.tcbf_group_execute_noalloc(1, tcbf.F16, 0, arr, 1, None) != 0            # not the current device
    ws = torch.empty(tcbf.GROUP_WORKSPACE_BYTES, dtype=torch.uint8, device="cuda:0")
    assert L.tcbf_group_execute(1, tcbf.F16, 0, arr, 1, ws.data_ptr(), None) != 0    # not the current device
    # a rejected call leaves no HIP error behind for the caller's next launch
    # check (torch checks the runtime's last error after each of its kernels)
    t = torch.rand(64, device="cuda:0") + 1.0
    torch.cuda.synchronize()
    assert float(t.min()) >= 1.0
