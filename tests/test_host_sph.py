"""The SPH neighbour walk (host, C++): every pair with a nonzero symmetrised
kernel weight, i.e. closer than max(h_i, h_j), appears in its group's list
(brute force over all pairs), lists hold particles only, each once and in
ascending order, and bad arguments are rejected."""
import numpy as np
import pytest

import synth
import paper_1206_1199_amd as otoo


def _sorted_inputs(pos, h, tree):
    perm, pos32, mass32, cm = tree.export(4)
    return perm, pos[perm], h[perm]


@pytest.mark.parametrize("dist,g_max,mode", [("plummer", 64, otoo.GROUP_CHUNK), ("plummer", 17, otoo.GROUP_CELL),
                                             ("poly", 256, otoo.GROUP_CHUNK), ("uniform", 1, otoo.GROUP_CHUNK)])
def test_lists_hold_every_neighbour(dist, g_max, mode):
    if dist == "plummer":
        pos, m = synth.plummer(3000, seed=11)
    elif dist == "uniform":
        pos, m = synth.uniform_sphere(800, seed=12)
    else:
        pos, m, _, _ = synth.polytrope_pair(1500, seed=13)
    h = synth.knn_radius(pos, 24)
    tree = otoo.Tree(pos, m, n_crit=16)
    lists = tree.walk_sph(h, g_max=g_max, group_mode=mode)
    perm, xs, hs = _sorted_inputs(pos, h, tree)
    n = len(m)
    assert np.all(lists.n_cellent == 0)
    assert np.all(lists.list_idx < n)
    d2 = ((xs[:, None, :] - xs[None, :, :]) ** 2).sum(-1)
    # pairs at exactly r = h (the k-th neighbour that defines h) have weight 0
    need = d2 < (np.maximum(hs[:, None], hs[None, :]) * (1 - 1e-9)) ** 2
    for g in range(len(lists.group_off) - 1):
        a, b = lists.group_off[g], lists.group_off[g + 1]
        L = lists.list_idx[lists.list_off[g]:lists.list_off[g + 1]]
        assert np.all(np.diff(L) > 0)                         # ascending, no duplicates
        req = np.flatnonzero(need[a:b].any(axis=0))
        assert np.isin(req, L).all(), f"group {g} misses neighbours"
    assert lists.interactions == int(np.sum(np.diff(lists.group_off) * np.diff(lists.list_off)))


def test_lists_are_not_everything():
    pos, m = synth.uniform_sphere(5000, seed=14)
    h = synth.knn_radius(pos, 32)
    lists = otoo.Tree(pos, m, n_crit=16).walk_sph(h, g_max=64)
    assert lists.n_entries < 0.2 * len(m) * (len(lists.group_off) - 1)


def test_bad_arguments():
    pos, m = synth.plummer(100, seed=15)
    tree = otoo.Tree(pos, m, n_crit=16)
    h = np.full(100, 0.1)
    for bad in (np.zeros(100), np.full(100, np.nan), -h):
        with pytest.raises(otoo.OtooError):
            tree.walk_sph(bad)
    with pytest.raises(otoo.OtooError):
        tree.walk_sph(h, g_max=0)
    with pytest.raises(ValueError):
        tree.walk_sph(h[:50])
