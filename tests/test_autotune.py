"""Autotuner host logic (CPU): cache keys, cache file round trip, choice of
the fastest shape, and that tuning leaves the process-wide shape set."""

import pytest

from paper_2009_09500_amd import autotune, binding


class FakeSegs:
    """Stands in for a device tensor: the injected timer never touches it."""

    def __init__(self, n):
        self.shape = (n, 6)
        self.device = None


@pytest.fixture(autouse=True)
def default_tuning():
    binding.vox_set_tuning(None)
    yield
    binding.vox_set_tuning(None)


def test_key_buckets_segment_counts():
    k = autotune.key("MI355X", (2048, 2048, 2048), 4_194_304)
    assert k == "MI355X|2048x2048x2048|n~2^22"
    assert autotune.key("d", (64, 64, 64), 3_000_000) == autotune.key("d", (64, 64, 64), 4_000_000)
    assert autotune.key("d", (64, 64, 64), 1_000) != autotune.key("d", (64, 64, 64), 100_000)
    assert autotune.key("d", (64, 64, 64), 0).endswith("n~2^-1")


def test_every_shape_is_compiled():
    for s in autotune.SHAPES:
        binding.vox_set_tuning(s)
        assert binding.vox_get_tuning() == s


def test_best_shape_and_ties():
    assert autotune.best_shape({(8, 6, 5): 2.0, (8, 6, 6): 1.0, (7, 6, 6): 3.0}) == (8, 6, 6)
    assert autotune.best_shape({(7, 7, 6): 1.0, (8, 6, 5): 1.0}) == (8, 6, 5)


def test_tune_caches_and_applies(tmp_path):
    cache = autotune.TuneCache(str(tmp_path / "t.json"))
    fake = {(8, 6, 5): 1.5, (8, 6, 6): 1.2, (7, 6, 6): 1.9, (7, 7, 6): 1.3}
    best, times = autotune.tune_grid(FakeSegs(1 << 20), (1024, 1024, 1024), cache=cache,
                                     timer=lambda s: fake[s], device="gfx950-test")
    assert best == (8, 6, 6) and times == fake
    assert binding.vox_get_tuning() == (8, 6, 6)
    again = autotune.TuneCache(str(tmp_path / "t.json"))          # reloaded from disk
    assert again.get(autotune.key("gfx950-test", (1024, 1024, 1024), 1 << 20)) == (8, 6, 6)
    binding.vox_set_tuning(None)
    assert autotune.apply((1024, 1024, 1024), 1 << 20, "gfx950-test", cache=again) == (8, 6, 6)
    assert binding.vox_get_tuning() == (8, 6, 6)
    binding.vox_set_tuning(None)
    assert autotune.apply((512, 512, 512), 1 << 20, "gfx950-test", cache=again) is None
    assert binding.vox_get_tuning() == (0, 0, 0)


def test_tuning_restored_when_timer_fails(tmp_path):
    binding.vox_set_tuning((7, 6, 6))
    cache = autotune.TuneCache(str(tmp_path / "t.json"))

    def boom(s):
        raise RuntimeError("timer failed")
    with pytest.raises(RuntimeError):
        autotune.tune_grid(FakeSegs(10), (64, 64, 64), cache=cache, timer=boom, device="x")
    assert binding.vox_get_tuning() == (7, 6, 6)


def test_corrupt_cache_is_ignored(tmp_path):
    p = tmp_path / "bad.json"
    p.write_text("{not json")
    assert autotune.TuneCache(str(p)).entries == {}
    p.write_text('{"k": {"shape": [9, 9, 9], "ms": {}}}')
    assert autotune.TuneCache(str(p)).get("k") is None
