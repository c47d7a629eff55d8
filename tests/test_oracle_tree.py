"""Pins of the oracle tree, its cell moments and its group walk.

* the paper's worked two-particle example (Eq. (3)) fixes b_max and B2;
* the absolute MAC radius (Eq. (1)) has the asymptotes the paper states;
* the walk partitions all particles for every group, degenerates to the
  full particle list at theta = 0 and never accepts a cell that holds a group
  particle;
* list sums over the walk's lists equal the direct sum at theta = 0 and stay
  within 1e-3 median of it at theta = 0.5, the error shrinking with theta.
"""
import math
import os

import numpy as np
import pytest

import oracle
import synth
from oracle import tree as otree
from tests.o3_helpers import o3_csr

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_eq3_two_particle_example():
    rows = np.loadtxt(os.path.join(GOLDEN, "eq3_two_particle.txt"))
    for m, L, bmax_ref, b2_ref in rows:
        pos = np.array([[0.0, 0.0, 0.0], [L, 0.0, 0.0]])
        tr = otree.build(pos, np.array([m, m]), n_crit=16)
        root = tr.root
        assert root.leaf
        assert root.b_max == pytest.approx(bmax_ref, rel=1e-15)
        assert np.trace(root.S) == pytest.approx(b2_ref, rel=1e-14)


def test_sw_radius_asymptotes():
    # m = L = 1: b_max = 1/2, B2 = 1/2 (Eq. (3)); r_b -> b_max for large Delta
    # and r_b ~ Delta^-1/4 for small Delta (Sec. 2.2)
    assert otree.sw_radius(0.5, 0.5, 1e12) == pytest.approx(0.5, rel=1e-5)
    d1, d2 = 1e-10, 1e-11
    slope = math.log(otree.sw_radius(0.5, 0.5, d2) / otree.sw_radius(0.5, 0.5, d1)) / math.log(d2 / d1)
    assert slope == pytest.approx(-0.25, abs=2e-3)
    # printed form with the corrected L^2/16 term, m = L = 1
    for delta in (0.1, 0.01, 0.001):
        ref = 0.25 + math.sqrt(1.0 / 16.0 + math.sqrt(1.5 / delta))
        assert otree.sw_radius(0.5, 0.5, delta) == pytest.approx(ref, rel=1e-15)


@pytest.fixture(scope="module")
def plummer_tree():
    pos, m = synth.plummer(4096, seed=0)
    tr = otree.build(pos, m, n_crit=16)
    return pos, m, tr


def test_cell_moments(plummer_tree):
    pos, m, tr = plummer_tree
    for c in tr.cells[:200]:
        assert c.M == pytest.approx(m[c.idx].sum(), rel=1e-14)
        if c.leaf:
            assert len(c.idx) <= 16 or c.level == 21
            continue
        # children partition the parent; parallel-axis theorem for S
        kids = np.concatenate([k.idx for k in c.children])
        assert np.array_equal(np.sort(kids), np.sort(c.idx))
        S = sum(k.S + k.M * np.outer(k.com - c.com, k.com - c.com) for k in c.children)
        np.testing.assert_allclose(S, c.S, rtol=1e-10, atol=1e-14 * np.abs(c.S).max())
        # every particle lies inside its cube
        p = pos[c.idx]
        assert np.all(np.abs(p - c.centre) <= c.side / 2 * (1 + 1e-12))


@pytest.mark.parametrize("theta", [0.0, 0.5, 0.9])
def test_walk_partition_and_no_self_cell(plummer_tree, theta):
    pos, m, tr = plummer_tree
    groups = otree.cell_groups(tr, 64)
    assert np.array_equal(np.sort(np.concatenate(groups)), np.arange(len(pos)))
    for g in groups[::7]:
        cells, parts = otree.walk(tr, pos, g, theta)
        covered = np.concatenate([np.asarray(parts, np.int64)] + [c.idx for c in cells])
        assert np.array_equal(np.sort(covered), np.arange(len(pos)))   # each particle exactly once
        gs = set(int(i) for i in g)
        for c in cells:
            assert not gs.intersection(int(i) for i in c.idx)
        assert gs.issubset(parts)
        if theta == 0.0:
            assert not cells


def _tree_error(pos, m, tr, theta, eps, sample):
    groups = otree.cell_groups(tr, 64)
    csr = o3_csr(tr, pos, groups, theta)
    order = csr["order"]
    inv = np.empty(len(order), np.int64)
    inv[order] = np.arange(len(order))
    acc, pot = oracle.list_force(pos[order], m[order], csr["group_off"], csr["list_off"],
                                 csr["list_idx"], csr["cell_com"], csr["cell_mass"], eps,
                                 tgt=inv[sample])
    acc0, pot0 = oracle.direct(pos, m, eps, tgt=sample)
    return oracle.rel_err(acc, acc0), oracle.rel_err(pot, pot0)


def test_theta0_lists_equal_direct(plummer_tree):
    pos, m, tr = plummer_tree
    sample = synth.sample_idx(len(pos), 256, seed=100)
    ea, ep = _tree_error(pos, m, tr, 0.0, 0.01, sample)
    assert ea.max() <= 1e-13 and ep.max() <= 1e-13


def test_tree_accuracy_vs_direct(plummer_tree):
    pos, m, tr = plummer_tree
    sample = synth.sample_idx(len(pos), 512, seed=100)
    med = []
    for theta in (0.3, 0.5, 0.8):
        ea, ep = _tree_error(pos, m, tr, theta, 0.01, sample)
        med.append(np.median(ea))
        if theta == 0.5:
            assert np.median(ea) <= 1e-3
            assert np.median(ep) <= 1e-3
    assert med[0] < med[1] < med[2]


def test_cell_groups_maximal(plummer_tree):
    pos, m, tr = plummer_tree
    for g in otree.cell_groups(tr, 64):
        assert 1 <= len(g) <= 64
