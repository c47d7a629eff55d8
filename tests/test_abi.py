"""The C ABI: every function include/otoo.h declares is exported by libotoo.so,
and the entry points reject bad arguments without touching a GPU."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_1206_1199_amd as otoo

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "otoo.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(otoo_[a-z_]+)\s*\(", txt)))


def test_every_declared_symbol_is_exported():
    lib = otoo.lib()
    names = _declared()
    assert len(names) >= 20
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(otoo.EXPORTED)


def test_null_context_and_bad_arguments_return_einval():
    lib = otoo.lib()
    assert lib.otoo_force(None, 1, None, None, 1, None, 0, None, None, 0, None, 4, 0.1, None, None,
                          None) == otoo.EINVAL
    assert lib.otoo_correction(None, 1, None, 1, None, 1, None, 0, None, None, 0, None, 0, None, 12, 0.1, None,
                               None) == otoo.EINVAL
    assert lib.otoo_quad_exact(None, 1, 1, 0, None, None, 0, None, 0, None, 12, None) == otoo.EINVAL
    assert lib.otoo_direct(None, 1, None, None, 0, None, 0.1, None, None) == otoo.EINVAL
    assert lib.otoo_sph_sum(None, 1, None, None, None, 1, None, 0, None, None, None) == otoo.EINVAL
    assert lib.otoo_tree_walk_sph(None, None, 0, 64, None) == otoo.EINVAL
    assert lib.otoo_tree_groups(None, 0, 64, None) == otoo.EINVAL
    assert lib.otoo_tree_walk_range(None, None, 0, 1, None) == otoo.EINVAL
    assert lib.otoo_check(None) == otoo.EINVAL
    assert lib.otoo_graph_launch(None) == otoo.EINVAL
    assert lib.otoo_autotune(None, None, None, None, 1, None, 1, 0.1, 1, None, None, None, None,
                             None) == otoo.EINVAL
    assert lib.otoo_set_tuning(None, None) == otoo.EINVAL
    assert lib.otoo_set_scratch_limit(None, 0) == otoo.EINVAL
    assert lib.otoo_last_error(None) == b"null context"
    assert lib.otoo_tree_build(None, None, 0, 16, None) == otoo.EINVAL
    assert lib.otoo_tree_walk(None, None, None) == otoo.EINVAL
