"""Host logic of the tile autotuner: cache keys, the choice rule and the JSON cache."""
import json

import clot_inputs as ci
from paper_2304_09180_amd import autotune, clot


def test_shape_key_is_a_multiset_of_channel_shapes():
    a = [ci.channel(2, 64, 16), ci.channel(2, 128, 32), ci.channel(2, 64, 16, seed=3)]
    b = [a[2], a[1], a[0]]
    assert autotune.shape_key(a) == autotune.shape_key(b) == "2d:128x32x1*1,64x16x1*2"
    assert autotune.shape_key([ci.channel(3, 32, 8, 8)]) == "3d:32x8x8*1"
    k32 = autotune.cache_key(a, clot.FP32_MIXED, "gfx950")
    k64 = autotune.cache_key(a, clot.FP64, "gfx950")
    assert k32.startswith("gfx950|fp32|") and k64.startswith("gfx950|fp64|") and k32 != k64


def test_choice_prefers_the_smaller_tile_within_one_percent():
    assert autotune.choose({256: 10.0, 512: 9.0, 1024: 9.5}) == 512
    assert autotune.choose({256: 10.0, 512: 9.95, 1024: 9.92}) == 256
    assert autotune.choose({256: 10.0, 512: 9.95, 1024: 9.0}) == 1024
    assert autotune.choose({512: 3.0}) == 512


def test_cache_round_trip_keeps_other_entries(tmp_path):
    path = str(tmp_path / "sub" / "tune.json")
    assert autotune.load_cache(path) == {}
    autotune.store_cache(path, "k1", {"tile": 256})
    autotune.store_cache(path, "k2", {"tile": 512})
    data = json.load(open(path))
    assert data == {"k1": {"tile": 256}, "k2": {"tile": 512}}
    (tmp_path / "bad.json").write_text("not json")
    assert autotune.load_cache(str(tmp_path / "bad.json")) == {}
