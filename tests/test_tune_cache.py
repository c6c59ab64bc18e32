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
