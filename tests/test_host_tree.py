"""Production host tree and walk (libotoo.so, C++/OpenMP) against the oracle tree.

The two trees are built independently (integer Hilbert keys vs recursive
geometric splits); they must agree cell by cell (same cubes, same particle
sets, same moments) and the walks must produce the same interaction lists
as sets, for both group modes and both acceptance criteria.
"""
import math

import numpy as np
import pytest

import synth
import paper_1206_1199_amd as otoo
from oracle import tree as otree


@pytest.fixture(scope="module")
def trees():
    pos, m = synth.plummer(3000, seed=0)
    t = otoo.Tree(pos, m, n_crit=16)
    o = otree.build(pos, m, n_crit=16)
    return pos, m, t, o


def test_cells_match_oracle(trees):
    pos, m, t, o = trees
    perm, _, _, _ = t.export()
    assert np.array_equal(np.sort(perm), np.arange(len(pos)))
    c = t.cells()
    assert t.n_cells == len(o.cells)
    ocells = {cell.key: cell for cell in o.cells}
    for k in range(t.n_cells):
        key = (int(c["level"][k]),) + tuple(int(v) for v in c["ijk"][k])
        oc = ocells[key]
        ids = perm[c["first"][k]:c["first"][k] + c["count"][k]]
        assert np.array_equal(np.sort(ids), np.sort(oc.idx))
        assert c["mass"][k] == pytest.approx(oc.M, rel=1e-13)
        np.testing.assert_allclose(c["com"][k], oc.com, rtol=1e-12, atol=1e-14)
        S_o = np.array([oc.S[0, 0], oc.S[1, 1], oc.S[2, 2], oc.S[0, 1], oc.S[0, 2], oc.S[1, 2]])
        np.testing.assert_allclose(c["S6"][k], S_o, rtol=1e-9, atol=1e-12 * np.abs(S_o).max() + 1e-300)
        assert c["side"][k] == pytest.approx(oc.side, rel=1e-15)
        assert c["s"][k] == pytest.approx(oc.s, rel=1e-9, abs=1e-14)
        assert c["bmax"][k] == pytest.approx(oc.b_max, rel=1e-12)


def test_links_traverse_every_particle_once(trees):
    pos, m, t, o = trees
    nxt, more = t.links()
    n = t.n
    seen = []
    u = n  # root; rule (1): open every cell
    while u != -1:
        if u < n:
            seen.append(u)
            u = nxt[u]
        else:
            u = more[u]
    assert seen == list(range(n))
    # next of the root is null, every cell has a more pointer
    assert nxt[n] == -1 and np.all(more[n:] >= 0)


def _prod_sets(t, lists, perm, cells, g):
    lo, hi = lists.list_off[g], lists.list_off[g + 1]
    ent = lists.list_idx[lo:hi]
    nce = lists.n_cellent[g]
    assert np.all(ent[:nce] >= t.n) and np.all(ent[nce:] < t.n)
    assert np.all(np.diff(ent[:nce]) > 0) and np.all(np.diff(ent[nce:]) > 0)
    ckeys = {(int(cells["level"][e - t.n]),) + tuple(int(v) for v in cells["ijk"][e - t.n]) for e in ent[:nce]}
    parts = set(int(perm[e]) for e in ent[nce:])
    return ckeys, parts


@pytest.mark.parametrize("mode,theta,mac", [(otoo.GROUP_CELL, 0.5, "bh"), (otoo.GROUP_CHUNK, 0.5, "bh"),
                                            (otoo.GROUP_CHUNK, 0.0, "bh"), (otoo.GROUP_CELL, 0.8, "bh"),
                                            (otoo.GROUP_CHUNK, 0.0, "sw")])
def test_walk_lists_equal_oracle_sets(trees, mode, theta, mac):
    pos, m, t, o = trees
    perm, _, _, _ = t.export()
    cells = t.cells()
    kw = dict(mac=otoo.MAC_ABSOLUTE, delta=1e-3, m_limit=0.05) if mac == "sw" else {}
    lists = t.walk(theta=theta, g_max=64, group_mode=mode, **kw)
    assert lists.group_off[0] == 0 and lists.group_off[-1] == t.n
    sizes = np.diff(lists.group_off)
    assert np.all((sizes >= 1) & (sizes <= 64))
    if mode == otoo.GROUP_CELL:
        # same groups as sets (the production order is the Hilbert order)
        og = {tuple(g) for g in otree.cell_groups(o, 64)}
        assert len(og) == lists.n_groups
    inter = 0
    for g in range(lists.n_groups):
        ids = perm[lists.group_off[g]:lists.group_off[g + 1]]
        if mode == otoo.GROUP_CELL:
            assert tuple(np.sort(ids)) in og
        okw = dict(mac="sw", delta=1e-3, m_limit=0.05) if mac == "sw" else {}
        oc, op = otree.walk(o, pos, ids, theta, **okw)
        ckeys, parts = _prod_sets(t, lists, perm, cells, g)
        assert ckeys == {c.key for c in oc}
        assert parts == set(op)
        assert set(int(i) for i in ids) <= parts          # self pairs present
        inter += len(ids) * (lists.list_off[g + 1] - lists.list_off[g])
    assert inter == lists.interactions


@pytest.mark.parametrize("mode,theta", [(otoo.GROUP_CHUNK, 0.7), (otoo.GROUP_CELL, 0.9), (otoo.GROUP_CHUNK, 0.0)])
def test_near_cells_listed_first_match_oracle(trees, mode, theta):
    """A walk with a near ratio lists, per group, the same entries as the
    plain walk; its cells are split into the near ones (side >= ratio x the
    distance of the COM from the group's box centre, the oracle's
    near_cells) and the others, each part ascending, n_near counting the
    first part; the (group, cell) pairs are the near cells."""
    pos, m, t, o = trees
    perm, _, _, _ = t.export()
    cells = t.cells()
    plain = t.walk(theta=theta, g_max=64, group_mode=mode)
    near = t.walk(theta=theta, g_max=64, group_mode=mode, near_ratio=0.4)
    np.testing.assert_array_equal(plain.group_off, near.group_off)
    np.testing.assert_array_equal(plain.list_off, near.list_off)
    np.testing.assert_array_equal(plain.n_cellent, near.n_cellent)
    assert np.all(plain.n_near == 0) and np.all(near.n_near <= near.n_cellent)
    np.testing.assert_array_equal(near.pair_off, np.concatenate([[0], np.cumsum(near.n_near)]))
    total_near = 0
    for g in range(near.n_groups):
        lo, hi = near.list_off[g], near.list_off[g + 1]
        a, b = near.list_idx[lo:hi], plain.list_idx[lo:hi]
        nce, nn = near.n_cellent[g], near.n_near[g]
        np.testing.assert_array_equal(a[nce:], b[nce:])                 # particles unchanged
        assert set(a[:nce].tolist()) == set(b[:nce].tolist())          # the same cells
        assert np.all(np.diff(a[:nn]) > 0) and np.all(np.diff(a[nn:nce]) > 0)
        ids = perm[near.group_off[g]:near.group_off[g + 1]]
        oc, _ = otree.walk(o, pos, ids, theta)
        want = {c.key for c in otree.near_cells(oc, pos, ids, 0.4)}
        got = {(int(cells["level"][e - t.n]),) + tuple(int(v) for v in cells["ijk"][e - t.n]) for e in a[:nn]}
        assert got == want
        total_near += nn
    assert (total_near > 0) == (theta > 0)


def test_theta_zero_lists_all_particles(trees):
    pos, m, t, o = trees
    lists = t.walk(theta=0.0, g_max=128)
    assert np.all(lists.n_cellent == 0)
    assert np.all(np.diff(lists.list_off) == t.n)


def test_depth_cap_and_duplicates():
    # many coincident particles force leaves at the depth cap larger than n_crit
    rng = np.random.default_rng(0)
    pos = np.vstack([np.zeros((300, 3)), rng.normal(size=(200, 3))])
    m = np.full(500, 1 / 500)
    t = otoo.Tree(pos, m, n_crit=8)
    lists = t.walk(theta=0.6, g_max=64, group_mode=otoo.GROUP_CELL)
    sizes = np.diff(lists.group_off)
    assert sizes.sum() == 500 and sizes.max() <= 64
    assert t.depth == 21


def test_host_entry_points_reject_bad_arguments():
    with pytest.raises(otoo.OtooError):
        otoo.Tree(np.zeros((0, 3)), np.zeros(0))
    with pytest.raises(otoo.OtooError):
        otoo.Tree(np.array([[0.0, math.nan, 0.0]]), np.ones(1))
    t = otoo.Tree(np.random.default_rng(1).normal(size=(100, 3)), np.ones(100))
    for kw in (dict(theta=1.2), dict(theta=-0.1), dict(g_max=0), dict(g_max=257), dict(group_mode=7),
               dict(mac=otoo.MAC_ABSOLUTE, delta=0.0)):
        with pytest.raises(otoo.OtooError):
            t.walk(**kw)


@pytest.mark.parametrize("mode,g_max", [(otoo.GROUP_CHUNK, 64), (otoo.GROUP_CELL, 100)])
def test_walk_in_batches_equals_whole_walk(mode, g_max):
    """Walking groups [g0, g1) batch by batch gives exactly the whole walk's
    lists (absolute group offsets, each batch's list offsets from 0)."""
    pos, m = synth.plummer(20000, seed=31)
    tree = otoo.Tree(pos, m, n_crit=16)
    whole = tree.walk(theta=0.6, g_max=g_max, group_mode=mode)
    G = tree.n_groups(g_max, mode)
    assert G == whole.n_groups
    edges = [0, 1, G // 3, G // 3 + 1, G - 5, G]
    go, lo, li, nc, inter = [0], [0], [], [], 0
    for a, b in zip(edges[:-1], edges[1:]):
        part = tree.walk_range(a, b, theta=0.6, g_max=g_max, group_mode=mode)
        assert part.n_groups == b - a and part.list_off[0] == 0
        assert part.group_off[0] == whole.group_off[a] and part.group_off[-1] == whole.group_off[b]
        go += list(part.group_off[1:])
        lo += list(part.list_off[1:] + lo[-1])
        li.append(part.list_idx)
        nc.append(part.n_cellent)
        inter += part.interactions
    np.testing.assert_array_equal(go, whole.group_off)
    np.testing.assert_array_equal(lo, whole.list_off)
    np.testing.assert_array_equal(np.concatenate(li), whole.list_idx)
    np.testing.assert_array_equal(np.concatenate(nc), whole.n_cellent)
    assert inter == whole.interactions
    # g_end past the group count is clamped; empty or out-of-range batches are rejected
    assert tree.walk_range(G - 2, G + 100, theta=0.6, g_max=g_max, group_mode=mode).n_groups == 2
    for a, b in ((5, 5), (-1, 3), (G, G + 1)):
        with pytest.raises(otoo.OtooError):
            tree.walk_range(a, b, theta=0.6, g_max=g_max, group_mode=mode)
