"""Pins of the FP64 direct sum (oracle_direct) and the Plummer generator.

Each value below is either worked out by hand (two bodies, cube corners),
an invariant of exact pairwise forces (momentum, angular momentum, the
virial identity that ties the acceleration to the potential), or the
closed-form potential of the Plummer sphere.
"""
import math

import numpy as np
import pytest
from scipy import integrate

import oracle
import synth


def test_two_body_hand_values():
    # m1 = 2 at the origin, m2 = 3 at (1, 2, 2): |d| = 3.
    pos = np.array([[0.0, 0.0, 0.0], [1.0, 2.0, 2.0]])
    m = np.array([2.0, 3.0])
    # eps = 4: r^2 + eps^2 = 25, (25)^(3/2) = 125, (25)^(1/2) = 5
    acc, pot = oracle.direct(pos, m, 4.0)
    np.testing.assert_allclose(acc[0], [0.024, 0.048, 0.048], rtol=1e-15)
    np.testing.assert_allclose(acc[1], [-0.016, -0.032, -0.032], rtol=1e-15)
    np.testing.assert_allclose(pot, [-0.6, -0.4], rtol=1e-15)
    # eps = 0: |d|^3 = 27
    acc, pot = oracle.direct(pos, m, 0.0)
    np.testing.assert_allclose(acc[0], [1 / 9, 2 / 9, 2 / 9], rtol=1e-15)
    np.testing.assert_allclose(acc[1], [-2 / 27, -4 / 27, -4 / 27], rtol=1e-15)
    np.testing.assert_allclose(pot, [-1.0, -2 / 3], rtol=1e-15)


def test_cube_corners_closed_form():
    # unit masses on the corners of the cube [-1, 1]^3: by symmetry every
    # force points to the centre; per axis it is
    #   -(1/4 + 1/(4 sqrt 2) + 1/(12 sqrt 3))  (3 edges, 3 face and 1 body diagonal)
    # and the potential is -(3/2 + 3/(2 sqrt 2) + 1/(2 sqrt 3)).
    corners = np.array([[sx, sy, sz] for sx in (-1, 1) for sy in (-1, 1) for sz in (-1, 1)], float)
    acc, pot = oracle.direct(corners, np.ones(8), 0.0)
    f = 0.25 + 1 / (4 * math.sqrt(2)) + 1 / (12 * math.sqrt(3))
    np.testing.assert_allclose(acc, -f * corners, rtol=1e-14)
    np.testing.assert_allclose(pot, -(1.5 + 1.5 / math.sqrt(2) + 0.5 / math.sqrt(3)), rtol=1e-14)


@pytest.mark.parametrize("eps", [0.0, 0.05])
def test_momentum_and_torque_vanish(eps):
    rng = np.random.default_rng(7)
    pos = rng.normal(size=(300, 3))
    m = rng.uniform(0.5, 2.0, 300)
    acc, _ = oracle.direct(pos, m, eps)
    scale = np.sum(m[:, None] * np.abs(acc))
    assert np.all(np.abs((m[:, None] * acc).sum(axis=0)) <= 1e-13 * scale)
    torque = (m[:, None] * np.cross(pos, acc)).sum(axis=0)
    assert np.all(np.abs(torque) <= 1e-13 * scale * np.abs(pos).max())


def test_virial_identity_links_acc_and_pot():
    # for unsoftened pair forces: sum_i m_i x_i . a_i = W = 1/2 sum_i m_i phi_i
    rng = np.random.default_rng(11)
    pos = rng.uniform(-1, 1, size=(400, 3))
    m = rng.uniform(0.1, 1.0, 400)
    acc, pot = oracle.direct(pos, m, 0.0)
    lhs = np.sum(m * np.einsum("ij,ij->i", pos, acc))
    w = 0.5 * np.sum(m * pot)
    assert abs(lhs - w) <= 1e-12 * abs(w)


def _plummer_phi(r, x_max):
    r_cut = 1.0 / math.sqrt(x_max ** (-2.0 / 3.0) - 1.0)
    return (-(1.0 + r * r) ** -0.5 + (1.0 + r_cut * r_cut) ** -1.5) / x_max


@pytest.mark.parametrize("n", [4096, 16384])
def test_plummer_potential_closed_form(n):
    # truncated Plummer sphere (G = M = a = 1, enclosed mass fraction cut at
    # x_max): phi(r) = [-(1 + r^2)^-1/2 + (1 + R_cut^2)^-3/2] / x_max.
    x_max = 0.999
    pos, m = synth.plummer(n, seed=0, x_max=x_max)
    _, pot = oracle.direct(pos, m, 0.01)
    r = np.linalg.norm(pos, axis=1)
    rel = np.abs(pot - _plummer_phi(r, x_max)) / np.abs(_plummer_phi(r, x_max))
    assert np.median(rel) <= 3.0 / math.sqrt(n)
    # total potential energy against the closed form integrated over the
    # mass profile dM = 3 r^2 (1 + r^2)^-5/2 dr / x_max
    r_cut = 1.0 / math.sqrt(x_max ** (-2.0 / 3.0) - 1.0)
    w_ref = 0.5 * integrate.quad(
        lambda s: _plummer_phi(s, x_max) * 3 * s * s * (1 + s * s) ** -2.5 / x_max, 0, r_cut)[0]
    w = 0.5 * np.sum(m * pot)
    assert abs(w - w_ref) / abs(w_ref) <= 5.0 / math.sqrt(n)
    # untruncated limit of W is -3 pi / 32
    assert abs(w_ref + 3 * math.pi / 32) < 0.01


def test_plummer_mass_profile():
    from scipy import stats
    x_max = 0.999
    pos, _ = synth.plummer(20000, seed=3, x_max=x_max, recentre=False)
    r = np.linalg.norm(pos, axis=1)
    cdf = lambda s: s ** 3 * (1 + s * s) ** -1.5 / x_max
    assert stats.kstest(r, cdf).pvalue > 1e-3
