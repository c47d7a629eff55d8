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

    def autotune(self, tree, eps, choices, schedules, reps=10, theta=0.5):
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
