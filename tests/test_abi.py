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
    assert lib.otoo_correction(None, 1, None, 1, None, 1, None, None, 0, None, None, 0, None, 0, None, 12, 0.1,
                               None, None) == otoo.EINVAL
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
    assert lib.otoo_scratch_generation(None, None) == otoo.EINVAL


def test_force_plan_checks_the_queue_range_on_the_host():
    """The size checks and scratch plan of otoo_force run on the host alone
    (the same function otoo_force calls before it touches the device): a call
    whose work items, plus one last queue fetch per persistent workgroup,
    would reach 2^31 is refused, since the device queue head, the item table
    and the longest-first order are 32-bit."""
    lib = otoo.lib()
    # 2^30 particles in 2^30 one-particle groups with 2^37 list entries in
    # chunks of 64: 2^30 + 2^31 items
    with pytest.raises(otoo.OtooError) as e:
        otoo.force_plan(1 << 30, 1 << 30, 1 << 37, 0, 64, 2048)
    assert e.value.code == otoo.EINVAL
    # just below the limit: items = n_groups + n_entries // chunk + 1
    wg = 2048
    n_groups = 1 << 20
    entries = (2 ** 31 - 1 - wg - n_groups - 2) * 64
    assert otoo.force_plan(1 << 30, n_groups, entries, 0, 64, wg) > 0
    with pytest.raises(otoo.OtooError):
        otoo.force_plan(1 << 30, n_groups, entries + 64, 0, 64, wg)
    # the other checks of otoo_force's sizes
    for args in ((0, 1, 0, 0, 1024, 1), (10, 11, 0, 0, 1024, 1), (10, 1, -1, 0, 1024, 1), (10, 1, 0, -1, 1024, 1),
                 (10, 1, 0, 0, 32, 1), (10, 1, 0, 0, 1024, 0)):
        assert lib.otoo_force_plan(*args, None) == otoo.EINVAL, args
    # the scratch holds at least the unified source table
    n, nc = 16384, 2500
    assert otoo.force_plan(n, 256, 400000, nc, 1024, 2048) >= 16 * (n + nc)


def test_noalloc_entry_point_checks_and_limit():
    """otoo_force_noalloc rejects a null context like otoo_force; its array
    size in the header is the binding's; and the scratch plan of the shapes
    it serves fits (a 2^20 Plummer-sized call) while a 4M-particle call does
    not (otoo_force_noalloc refuses such a call before it enqueues)."""
    lib = otoo.lib()
    assert lib.otoo_force_noalloc(None, 1, None, None, 1, None, 0, None, None, 0, None, 4, 0.1, None, None,
                                  None) == otoo.EINVAL
    txt = open(os.path.join(ROOT, "include", "otoo.h")).read()
    m = re.search(r"#define OTOO_NOALLOC_SCRATCH_BYTES \((\d+) \* (\d+) \* (\d+)\)", txt)
    assert m and int(m.group(1)) * int(m.group(2)) * int(m.group(3)) == otoo.NOALLOC_SCRATCH_BYTES
    # Plummer 2^20, groups of 64, ~8e7 list entries, ~2.4e5 cells, chunk 16384, 8 workgroups per CU
    assert otoo.force_plan(1 << 20, 1 << 14, 81_386_028, 241_881, 16384, 2048) <= otoo.NOALLOC_SCRATCH_BYTES
    assert otoo.force_plan(1 << 22, 1 << 16, 330_000_000, 970_000, 16384, 2048) > otoo.NOALLOC_SCRATCH_BYTES
