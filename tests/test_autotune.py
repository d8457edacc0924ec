"""Autotuner host logic (CPU): cache keys, cache file round trip, choice of
the fastest candidate, and that the choice lands in the library's autotune
cache for its volume and segment count only."""

import pytest

from paper_2009_09500_amd import autotune, binding


class FakeSegs:
    """Stands in for a device tensor: the injected timer never touches it."""

    def __init__(self, n):
        self.shape = (n, 6)
        self.device = None


@pytest.fixture(autouse=True)
def empty_cache():
    binding.vox_tuning_cache_clear()
    yield
    binding.vox_tuning_cache_clear()


def test_key_buckets_segment_counts():
    k = autotune.key("MI355X", (2048, 2048, 2048), 4_194_304)
    assert k == "MI355X|2048x2048x2048|n~2^22"
    assert autotune.key("d", (64, 64, 64), 3_000_000) == autotune.key("d", (64, 64, 64), 4_000_000)
    assert autotune.key("d", (64, 64, 64), 1_000) != autotune.key("d", (64, 64, 64), 100_000)
    assert autotune.key("d", (64, 64, 64), 0).endswith("n~2^-1")


def test_every_candidate_is_a_valid_tuning():
    for c in autotune.CANDIDATES:
        binding.vox_tuning_cache_set((512, 512, 512), 1 << 20, autotune.tuning_of(c))
        t = binding.vox_tuning_cache_get((512, 512, 512), 1 << 20)
        assert (tuple(t.brick_lg), t.fill_wgs_per_cu) == (c[:3], c[3])


def test_best_candidate_and_ties():
    assert autotune.best_candidate({(8, 6, 5, 2): 2.0, (8, 6, 6, 0): 1.0, (7, 6, 6, 1): 3.0}) == (8, 6, 6, 0)
    assert autotune.best_candidate({(7, 7, 6, 0): 1.0, (8, 6, 5, 2): 1.0}) == (8, 6, 5, 2)


def test_tune_caches_and_installs(tmp_path):
    cache = autotune.TuneCache(str(tmp_path / "t.json"))
    fake = {c: 1.5 + 0.1 * i for i, c in enumerate(autotune.CANDIDATES)}
    fake[(8, 6, 6, 0)] = 1.2
    best, times = autotune.tune_grid(FakeSegs(1 << 20), (1024, 1024, 1024), cache=cache,
                                     timer=lambda c: fake[c], device="gfx950-test")
    assert best == (8, 6, 6, 0) and times == fake
    t = binding.vox_tuning_cache_get((1024, 1024, 1024), 1 << 20)
    assert tuple(t.brick_lg) == (8, 6, 6) and t.fill_wgs_per_cu == 0
    # Other volumes and counts keep the default.
    assert binding.vox_tuning_cache_get((512, 512, 512), 1 << 20) is None
    assert binding.vox_tuning_cache_get((1024, 1024, 1024), 1 << 10) is None
    again = autotune.TuneCache(str(tmp_path / "t.json"))          # reloaded from disk
    assert again.get(autotune.key("gfx950-test", (1024, 1024, 1024), 1 << 20)) == (8, 6, 6, 0)
    binding.vox_tuning_cache_clear()
    assert autotune.apply((1024, 1024, 1024), 1 << 20, "gfx950-test", cache=again) == (8, 6, 6, 0)
    assert tuple(binding.vox_tuning_cache_get((1024, 1024, 1024), 1 << 20).brick_lg) == (8, 6, 6)
    assert autotune.apply((512, 512, 512), 1 << 20, "gfx950-test", cache=again) is None


def test_failed_timer_installs_nothing(tmp_path):
    cache = autotune.TuneCache(str(tmp_path / "t.json"))

    def boom(c):
        raise RuntimeError("timer failed")
    with pytest.raises(RuntimeError):
        autotune.tune_grid(FakeSegs(1 << 20), (64, 64, 64), cache=cache, timer=boom, device="x")
    assert binding.vox_tuning_cache_get((64, 64, 64), 1 << 20) is None


def test_corrupt_cache_is_ignored(tmp_path):
    p = tmp_path / "bad.json"
    p.write_text("{not json")
    assert autotune.TuneCache(str(p)).entries == {}
    p.write_text('{"k": {"candidate": [9, 9, 9, 0], "ms": {}}}')
    assert autotune.TuneCache(str(p)).get("k") is None
    p.write_text('{"k": {"shape": [8, 6, 6], "ms": {}}}')              # an older file's entry
    assert autotune.TuneCache(str(p)).get("k") is None
