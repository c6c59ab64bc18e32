"""Autotuner bookkeeping (no GPU): cache keys and the JSON cache round trip;
the seed of the fp16 sweep is the variant matching Table 3's MI300X point."""
import json

from paper_2505_03269_amd import BLOCKED, F16, INTERLEAVED, tune


def test_cache_key_distinguishes_every_field():
    base = tune.cache_key("gfx950", F16, 256, 1024, 4096, 576, kernel_set="abc")
    assert base == "gfx950|dtype0|256x1024x4096x576|c0|s0|ksabc"
    others = [tune.cache_key("gfx942", F16, 256, 1024, 4096, 576, kernel_set="abc"),
              tune.cache_key("gfx950", 2, 256, 1024, 4096, 576, kernel_set="abc"),
              tune.cache_key("gfx950", F16, 255, 1024, 4096, 576, kernel_set="abc"),
              tune.cache_key("gfx950", F16, 256, 1024, 4096, 577, kernel_set="abc"),
              tune.cache_key("gfx950", F16, 256, 1024, 4096, 576, INTERLEAVED, kernel_set="abc"),
              tune.cache_key("gfx950", F16, 256, 1024, 4096, 576, a_shared=True, kernel_set="abc"),
              tune.cache_key("gfx950", F16, 256, 1024, 4096, 576, operand_layout=BLOCKED, kernel_set="abc"),
              tune.cache_key("gfx950", F16, 256, 1024, 4096, 576, kernel_set="abd")]
    assert len(set(others + [base])) == len(others) + 1


def test_cache_key_names_the_built_kernel_set():
    """Without an explicit kernel set the key carries the built library's
    identity (library bytes and candidate lists), stable within a process."""
    k1 = tune.cache_key("gfx950", F16, 1, 8, 8, 8)
    assert k1 == tune.cache_key("gfx950", F16, 1, 8, 8, 8)
    assert k1.startswith("gfx950|dtype0|1x8x8x8|c0|s0|ks") and len(tune.kernel_set_id()) == 12


def test_cache_round_trip(tmp_path):
    p = str(tmp_path / "tune.json")
    assert tune.load_cache(p) == {}
    c = {"k": {"variant": 2, "ms": {"2": 1.5, "6": 1.7}, "seed": 2}}
    tune.save_cache(p, c)
    assert tune.load_cache(p) == c
    assert json.load(open(p)) == c


def test_fp16_sweep_starts_from_table3_point():
    assert tune.CANDIDATES[F16][0] == 2
    assert sorted(tune.CANDIDATES[F16]) == [1, 2, 3, 4, 5, 6, 7, 8, 9]


def test_group_variant_skips_the_generic_kernel():
    """The grouped launch has no generic-kernel form: a problem whose tuned
    plan is the generic kernel joins the group with its fastest other variant."""
    assert tune.group_variant({"variant": 9, "ms": {"2": 1.2, "9": 1.0}}) == 9
    assert tune.group_variant({"variant": 1, "ms": {"1": 0.9, "2": 1.3, "6": 1.1, "9": 1.2}}) == 6
    try:
        tune.group_variant({"variant": 1, "ms": {"1": 0.9}})
    except tune.TcbfError:
        pass
    else:
        raise AssertionError("a problem only the generic kernel takes has no grouped variant")


def test_group_variants_use_the_cache_per_shape(tmp_path, monkeypatch):
    """group_variants tunes each distinct shape once (cached entries are
    reused) and gives FP8 / 1-bit problems variant 0."""
    calls = []

    def fake_tune(batch, M, N, K, dtype, c_layout, a_shared, **kw):
        calls.append((batch, M, N, K, a_shared))
        return {"variant": 1 if N == 8 else 9, "ms": {"1": 1.0, "2": 2.0, "9": 3.0}}
    monkeypatch.setattr(tune, "tune", fake_tune)
    shapes = [(1, 64, 8, 64), (1, 64, 16, 64), (1, 64, 8, 64), (2, 64, 16, 64, 1)]
    assert tune.group_variants(shapes) == [2, 9, 2, 9]
    assert len(calls) == 3
    assert tune.group_variants(shapes, dtype=2) == [0, 0, 0, 0]


def test_tune_group_times_the_launch_and_caches(tmp_path, monkeypatch):
    """tune_group times each candidate variant list with the caller's grouped
    launch, keeps the fastest, times a list that two policies share once, and
    answers from its cache afterwards."""
    monkeypatch.setattr(tune, "group_variants", lambda shapes, *a, **k: [5] * len(shapes))
    monkeypatch.setattr(tune, "_accepts", lambda s, v, *a: s[2] >= 64)
    shapes = [(1, 256, 64, 128), (1, 128, 32, 64)]
    cost = {(0, 0): 3.0, (5, 5): 2.0, (9, 2): 1.0, (2, 2): 4.0}
    timed = []

    def measure(v):
        timed.append(tuple(v))
        return cost[tuple(v)]
    p = str(tmp_path / "t.json")
    e = tune.tune_group(shapes, measure, cache_path=p, arch="gfx950")
    assert e["variants"] == [9, 2] and e["policy"] == "ping_pong"
    assert sorted(timed) == sorted(cost) and e["ms"]["small_tiles"] == 4.0
    timed.clear()
    assert tune.tune_group(shapes, measure, cache_path=p, arch="gfx950") == e and not timed
    key = tune.group_cache_key("gfx950", F16, shapes)
    assert key in tune.load_cache(p) and "group[1x256x64x128,1x128x32x64]" in key
    assert tune.tune_group(shapes, measure, dtype=2, arch="gfx950")["variants"] == [0, 0]
