"""Autotuner bookkeeping (no GPU): cache keys and the JSON cache round trip;
the seed of the fp16 sweep is the variant matching Table 3's MI300X point."""
import json

from paper_2505_03269_amd import BLOCKED, F16, INTERLEAVED, tune


def test_cache_key_distinguishes_every_field():
    base = tune.cache_key("gfx950", F16, 256, 1024, 4096, 576)
    assert base == "gfx950|dtype0|256x1024x4096x576|c0|s0"
    others = [tune.cache_key("gfx942", F16, 256, 1024, 4096, 576), tune.cache_key("gfx950", 2, 256, 1024, 4096, 576),
              tune.cache_key("gfx950", F16, 255, 1024, 4096, 576), tune.cache_key("gfx950", F16, 256, 1024, 4096, 577),
              tune.cache_key("gfx950", F16, 256, 1024, 4096, 576, INTERLEAVED),
              tune.cache_key("gfx950", F16, 256, 1024, 4096, 576, a_shared=True),
              tune.cache_key("gfx950", F16, 256, 1024, 4096, 576, operand_layout=BLOCKED)]
    assert len(set(others + [base])) == len(others) + 1


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
