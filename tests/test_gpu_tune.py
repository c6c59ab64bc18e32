"""Autotuner on the device: it times every valid variant, caches the fastest
and hands back a plan that uses it."""
import numpy as np
import pytest

import workloads as wl
from gpu_util import log, to_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_2505_03269_amd as tcbf  # noqa: E402
from paper_2505_03269_amd import tune  # noqa: E402


def test_tune_picks_a_measured_variant_and_caches(tmp_path):
    path = str(tmp_path / "tune.json")
    e = tune.tune(2, 256, 256, 192, tcbf.F16, cache_path=path, reps=3, warmup=1)
    assert str(e["variant"]) in e["ms"] and e["seed"] == 2
    assert set(e["ms"]) == {"1", "2", "3", "4", "5", "6", "7", "8", "9"}
    assert e["ms"][str(e["variant"])] == min(e["ms"].values())
    cache = tune.load_cache(path)
    assert len(cache) == 1 and list(cache.values())[0] == e
    # a cached entry is used as is (no new timing)
    key = list(cache)[0]
    cache[key]["variant"] = 5
    tune.save_cache(path, cache)
    plan = tune.tuned_plan(2, 256, 256, 192, tcbf.F16, cache_path=path)
    assert plan.info()["variant"] == 5
    # and the tuned plan computes the same result as the default one
    W, X = wl.random_f16_case(3, 2, 256, 256, 192)
    A, B = to_dev(W), to_dev(X)
    C1 = plan.empty_output()
    plan.execute(A, B, C1)
    d = tcbf.Plan(2, 256, 256, 192, tcbf.F16)
    C2 = d.empty_output()
    d.execute(A, B, C2)
    torch.cuda.synchronize()
    assert np.array_equal(C1.cpu().numpy(), C2.cpu().numpy())


@pytest.mark.parametrize("dtype", [tcbf.F8_E4M3, tcbf.MXF8_E4M3, tcbf.INT1])
def test_tune_other_dtypes(tmp_path, dtype):
    e = tune.tune(1, 256, 256, 512, dtype, cache_path=str(tmp_path / "t.json"), reps=2, warmup=1)
    assert set(e["ms"]) == {"1", "2", "3"}
    if dtype == tcbf.MXF8_E4M3:
        # ceil(Kp / 64) = 9: the ping-pong kernel refuses per-block scales
        e = tune.tune(1, 256, 256, 576, dtype, cache_path=str(tmp_path / "t.json"), reps=2, warmup=1)
        assert set(e["ms"]) == {"1", "2"}


@pytest.mark.parametrize("dtype", [tcbf.F16, tcbf.F8_E4M3])
def test_tune_blocked_operands(tmp_path, dtype):
    """Blocked operands: only the variants that read them are timed, under
    their own cache key, and the tuned plan takes blocked tensors."""
    path = str(tmp_path / "tb.json")
    e = tune.tune(2, 256, 256, 192, dtype, cache_path=path, reps=2, warmup=1, operand_layout=tcbf.BLOCKED)
    want = {"2", "5", "6", "8", "9"} if dtype == tcbf.F16 else {"1", "2", "3"}
    assert set(e["ms"]) == want
    plan = tune.tuned_plan(2, 256, 256, 192, dtype, cache_path=path, operand_layout=tcbf.BLOCKED)
    assert plan.a_layout == tcbf.BLOCKED and plan.info()["variant"] == e["variant"]
    assert len(tune.load_cache(path)) == 1


def test_tune_group_output_equals_each_tuned_plan(tmp_path):
    """The grouped launch with the variants tune_group chose (by timing the
    launch itself) gives every problem the output of its own plan with that
    variant, bit for bit; the choice is cached under the group's shapes."""
    shapes = [(1, 300, 264, 576), (2, 128, 128, 64), (8, 1024, 512, 128), (3, 200, 392, 200),
              (1, 2048, 1024, 256)]
    cases = []
    for i, (b, M, N, K) in enumerate(shapes):
        W, X = wl.random_f16_case(300 + i, b, M, N, K)
        cases.append((to_dev(W), to_dev(X), torch.empty((b, 2, M, N), device="cuda:0")))
    ws = torch.zeros(tcbf.GROUP_WORKSPACE_BYTES, dtype=torch.uint8, device="cuda:0")

    def measure(v):
        for _ in range(2):
            tcbf.group_execute(cases, workspace=ws, variants=v)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(5):
            tcbf.group_execute(cases, workspace=ws, variants=v)
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / 5
    path = str(tmp_path / "g.json")
    ent = tune.tune_group(shapes, measure, cache_path=path, reps=2, warmup=1)
    log("group tuning: %s" % ent)
    assert set(ent["ms"]) == {"default", "per_problem", "ping_pong", "small_tiles"}
    assert ent["ms"][ent["policy"]] == min(ent["ms"].values())
    assert tune.tune_group(shapes, lambda v: 1 / 0, cache_path=path) == ent
    for (_, _, C) in cases:
        C.fill_(float("nan"))
    tcbf.group_execute(cases, workspace=ws, variants=ent["variants"])
    torch.cuda.synchronize()
    for v, (b, M, N, K), (Wd, Xd, C) in zip(ent["variants"], shapes, cases):
        plan = tcbf.Plan(b, M, N, K, tcbf.F16, variant=v)
        ref = plan.empty_output()
        plan.execute(Wd, Xd, ref)
        torch.cuda.synchronize()
        assert torch.equal(C, ref), (v, b, M, N, K)
