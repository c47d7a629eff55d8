"""OTOO_* environment overrides (host logic, no GPU): parsing, the walks'
default group size and the autotuner's cache path."""
import numpy as np
import pytest

import synth
import paper_1206_1199_amd as otoo
from paper_1206_1199_amd import autotune as at


def test_parsing():
    env = {"OTOO_CHUNK": "4096", "OTOO_TILE": " 1024 ", "OTOO_LPT": "0", "OTOO_GMAX": "", "OTHER": "x"}
    assert otoo.env_overrides(env) == {"chunk": 4096, "tile": 1024, "lpt": 0}
    assert otoo.env_overrides({}) == {}
    with pytest.raises(ValueError, match="OTOO_BLOCKS_PER_CU"):
        otoo.env_overrides({"OTOO_BLOCKS_PER_CU": "six"})


def test_walk_default_group_size(monkeypatch):
    pos, m = synth.plummer(2000, 21)
    t = otoo.Tree(pos, m)
    monkeypatch.delenv("OTOO_GMAX", raising=False)
    assert np.diff(t.walk(theta=0.5).group_off).max() == 64
    monkeypatch.setenv("OTOO_GMAX", "32")
    lists = t.walk(theta=0.5)
    assert np.diff(lists.group_off).max() == 32 and t.n_groups() == lists.n_groups
    assert np.diff(t.walk(theta=0.5, g_max=128).group_off).max() == 128   # an explicit argument wins


def test_autotune_cache_path():
    assert at.default_cache({"OTOO_AUTOTUNE_CACHE": "/tmp/x.json"}) == "/tmp/x.json"
    assert at.default_cache({}) == at.PACKAGE_CACHE
