"""Host logic of the batch-size autotuner: size classes, the choice rule and
the cache file (no GPU)."""
import os

from paper_1607_00908_amd import tune


def test_size_classes_split_at_the_bounds():
    assert tune.size_class(1) == 0
    assert tune.size_class(1 << 18) == 0
    assert tune.size_class((1 << 18) + 1) == 1
    assert tune.size_class(1 << 20) == 1
    assert tune.size_class(1 << 22) == 2
    assert tune.size_class(4096 * 4096) == 3


def test_choice_prefers_the_smaller_batch_within_tolerance():
    assert tune.choose({8: 100.0, 16: 80.0, 32: 79.0}) == 16
    assert tune.choose({8: 100.0, 16: 80.0, 32: 70.0}) == 32
    assert tune.choose({4: 50.0}) == 4
    assert tune.choose({32: 10.0, 64: 10.1}, tolerance=0.0) == 32


def test_cache_round_trip(tmp_path):
    p = os.path.join(tmp_path, "tune.json")
    c = tune.TuneCache(p)
    assert c.get("gfx950", 1 << 20) is None
    c.put("gfx950", 1 << 20, 32, {16: 40.0, 32: 35.5})
    c2 = tune.TuneCache(p)
    assert c2.get("gfx950", 1 << 20) == 32
    assert c2.get("gfx950", 1 << 19) == 32       # same class
    assert c2.get("gfx950", 1 << 24) is None
