"""The autotuner's choice among measured schedules (host logic, no GPU): the
fastest schedule wins unless another is within 1 % of its time and runs more
interactions per second."""
import numpy as np

from paper_1206_1199_amd import GROUP_CELL, GROUP_CHUNK
from paper_1206_1199_amd import autotune as at

GRID = {"group": [(GROUP_CHUNK, 64), (GROUP_CELL, 128)], "chunk": [2048, 16384], "blocks_per_cu": [4],
        "lpt": [1], "tile": [512]}


class _FakeContext:
    """Stands in for Context.autotune with given times [choice, schedule] and
    interaction counts [choice]."""

    def __init__(self, ms, inter):
        self.ms, self.inter = np.asarray(ms, np.float32), np.asarray(inter, np.int64)

    def sync_stream(self):
        pass

    def autotune(self, tree, eps, choices, schedules, reps=10, theta=0.5, corr_kind=-1, net=None, near_ratio=0.0):
        assert self.ms.shape == (len(choices), len(schedules))
        return self.ms, self.inter, None, None, None


def _pick(ms, inter):
    best, table = at.autotune(None, 0.005, 0.5, _FakeContext(ms, inter), grid=GRID)
    assert len(table) == 4
    return best["group_mode"], best["g_max"], best["chunk"]


def test_fastest_schedule_wins_outside_the_tie_band():
    # cell groups 2 % faster with fewer interactions: the time decides
    assert _pick([[1.70, 1.66], [1.70, 1.627]], [5.2e9, 4.5e9]) == ("cell", 128, 16384)


def test_tie_goes_to_the_higher_interaction_rate():
    # within 1 %: chunk 64 does 15 % more interactions in the same time
    assert _pick([[1.70, 1.638], [1.70, 1.637]], [5.2e9, 4.5e9]) == ("chunk", 64, 16384)
    # and inside one group choice the faster schedule of the two
    assert _pick([[1.640, 1.638], [1.90, 1.90]], [5.2e9, 4.5e9]) == ("chunk", 64, 16384)


def test_corrected_step_has_its_own_cache_entry(tmp_path, monkeypatch):
    """A corrected mode reads its own entry, falls back to the plain force's,
    and then to the defaults."""
    monkeypatch.setattr(at, "device_key", lambda device=0: "gfx950:256cu")
    path = str(tmp_path / "cache.json")
    plain = dict(group_mode="chunk", g_max=32, chunk=2048, blocks_per_cu=8, lpt=0, tile=512)
    learned = dict(group_mode="cell", g_max=256, chunk=4096, blocks_per_cu=6, lpt=1, tile=256)
    assert at.cached_schedule("cube16m", path=path, mode="learned") == (at.DEFAULT_SCHEDULE, "defaults")
    at.save_cache(at.cache_key("cube16m"), plain, path)
    sched, source = at.cached_schedule("cube16m", path=path, mode="learned")
    assert sched == plain and source == "autotune cache (plain force)"
    at.save_cache(at.cache_key("cube16m", "learned"), learned, path)
    sched, source = at.cached_schedule("cube16m", path=path, mode="learned")
    assert sched == learned and source == "autotune cache (learned step)"
    assert at.cached_schedule("cube16m", path=path) == (plain, "autotune cache")


def test_near_ratio_is_the_fastest_within_the_error_bound():
    """The learned step's near ratio: the fastest of the ratios whose measured
    median error holds the bound; with none holding it, the most accurate."""
    rows = [dict(near_ratio=0.4, ms=10.5, median_err=4.5e-4), dict(near_ratio=0.5, ms=8.5, median_err=6.9e-4),
            dict(near_ratio=0.6, ms=8.1, median_err=8.5e-4)]
    assert at.choose_near_ratio(rows, 1e-3)["near_ratio"] == 0.6
    assert at.choose_near_ratio(rows, 8e-4)["near_ratio"] == 0.5
    assert at.choose_near_ratio(rows, 5e-4)["near_ratio"] == 0.4
    assert at.choose_near_ratio(rows, 1e-4)["near_ratio"] == 0.4     # none holds it: the most accurate
    assert at.choose_near_ratio(rows[::-1], 1e-3)["near_ratio"] == 0.6


def test_learned_entry_carries_its_near_ratio(tmp_path, monkeypatch):
    monkeypatch.setattr(at, "device_key", lambda device=0: "gfx950:256cu")
    path = str(tmp_path / "cache.json")
    assert at.cached_near_ratio("cube16m", path=path, default=0.4) == 0.4
    entry = dict(group_mode="cell", g_max=256, chunk=16384, blocks_per_cu=6, lpt=0, tile=512, near_ratio=0.6,
                 median_err=8.5e-4, err_target=1e-3)
    at.save_cache(at.cache_key("cube16m", "learned"), entry, path)
    assert at.cached_near_ratio("cube16m", path=path, default=0.4) == 0.6
    sched, _ = at.cached_schedule("cube16m", path=path, mode="learned")
    assert "near_ratio" not in sched and sched["g_max"] == 256
