"""Pins of the input generators (textbook constants and closed forms)."""
import math

import numpy as np
import pytest

import oracle
import synth


def test_lane_emden_n15_constants():
    # tabulated n = 1.5 values: xi_1 = 3.65375, -xi_1^2 theta'(xi_1) = 2.71406,
    # rho_c / rho_mean = xi_1^3 / (3 * 2.71406) = 5.99071
    _, _, _, xi1, dth1 = synth.lane_emden(1.5)
    assert xi1 == pytest.approx(3.65375, abs=2e-5)
    assert -xi1 * xi1 * dth1 == pytest.approx(2.71406, abs=2e-5)
    assert xi1 ** 3 / (3 * -xi1 * xi1 * dth1) == pytest.approx(5.99071, abs=1e-4)


def test_polytrope_pair_energy_and_shell_theorem():
    n_each = 4096
    pos, m, star, centres = synth.polytrope_pair(n_each, seed=2)
    assert np.allclose((m[:, None] * pos).sum(0) / m.sum(), 0, atol=2e-3 * 0.05)
    # self-energy of an n-polytrope: W = -3/(5-n) M^2/R = -(6/7) M^2/R for n = 1.5
    for s, (M, R) in enumerate(((0.6, 0.02), (0.9, 0.012))):
        sel = star == s
        _, pot = oracle.direct(pos[sel], m[sel], 1e-5)
        w = 0.5 * np.sum(m[sel] * pot)
        assert w == pytest.approx(-(6 / 7) * M * M / R, rel=0.02)
    # the stars do not overlap: the pull of B on A's particles is that of a
    # point mass 0.9 at B's centre (shell theorem), up to sampling noise
    a_sel = np.where(star == 0)[0][:256]
    b_idx = np.where(star == 1)[0]
    src_off = np.arange(len(a_sel) + 1) * len(b_idx)
    a_b, _ = oracle.point_field(pos[a_sel], src_off, np.tile(b_idx, len(a_sel)), pos, m, 0.0)
    d = centres[1] - pos[a_sel]
    a_pt = 0.9 * d / (np.linalg.norm(d, axis=1) ** 3)[:, None]
    assert np.median(oracle.rel_err(a_b, a_pt)) < 5e-3


def test_grf_cube_lattice_and_rms():
    pos, m = synth.grf_cube(16, seed=4, rms=0.0)
    assert len(pos) == 16 ** 3 and m.sum() == pytest.approx(1.0)
    # the unperturbed lattice is mirror symmetric about the cube centre
    acc, _ = oracle.direct(pos, m, 1e-3)
    mirror = np.lexsort(((1 - pos)[:, 2], pos[:, 1], pos[:, 0]))
    key = np.lexsort((pos[:, 2], pos[:, 1], pos[:, 0]))
    refl = np.empty(len(pos), np.int64)
    refl[key] = mirror
    np.testing.assert_allclose(acc[refl, 2], -acc[:, 2], atol=1e-12 * np.abs(acc).max())
    p1, _ = synth.grf_cube(16, seed=4, rms=0.3)
    p2, _ = synth.grf_cube(16, seed=4, rms=0.3)
    assert np.array_equal(p1, p2) and not np.allclose(p1, pos)


def test_sample_idx_distinct_sorted():
    s = synth.sample_idx(1000, 100, seed=5)
    assert len(np.unique(s)) == 100 and np.all(np.diff(s) > 0)
