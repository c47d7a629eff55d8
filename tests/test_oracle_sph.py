"""Pins of the oracle's SPH gather sums (Sec. 2.3, Eq. 4; cubic B-spline kernel
of compact support h, symmetrised pair weight).

- hand values of W at u = r/h = 0, 1/2, 3/4, 1 from the spline's definition;
- the spline is C^1: value and slope agree on both sides of u = 1/2 and
  vanish at u = 1 (a wrong coefficient breaks one of these);
- normalisation: the volume integral of W is 1 for any h (quadrature);
- on a unit cubic lattice with unit masses and h = 2, 2.5, 3 the density of
  an interior particle is 1 to within the kernel's lattice error;
- two particles with different h: the hand value of the symmetrised sum.
"""
import math

import numpy as np
import pytest
from scipy import integrate

import oracle


def test_kernel_hand_values():
    for h in (0.5, 1.0, 3.0):
        s = 8.0 / (math.pi * h ** 3)
        assert oracle.sph_kernel(0.0, h) == pytest.approx(s, rel=1e-15)
        assert oracle.sph_kernel(0.5 * h, h) == pytest.approx(s / 4, rel=1e-14)      # 1 - 6/4 + 6/8
        assert oracle.sph_kernel(0.75 * h, h) == pytest.approx(s / 32, rel=1e-14)    # 2 (1/4)^3
        assert oracle.sph_kernel(h, h) == 0.0
        assert oracle.sph_kernel(1.7 * h, h) == 0.0


def test_kernel_is_c1():
    h, e = 1.3, 1e-6
    W = lambda u: oracle.sph_kernel(u * h, h)
    lo, hi = W(0.5 - e), W(0.5 + e)
    assert lo == pytest.approx(hi, abs=1e-5)
    slope_lo = (W(0.5 - e) - W(0.5 - 2 * e)) / e
    slope_hi = (W(0.5 + 2 * e) - W(0.5 + e)) / e
    assert slope_lo == pytest.approx(slope_hi, rel=1e-4)
    assert abs(W(1 - e)) < 1e-15 and abs((W(1 - e) - W(1 - 2 * e)) / e) < 1e-9   # (1 - u)^3 at u -> 1
    assert (W(e) - W(0)) / e == pytest.approx(0.0, abs=1e-4)                     # flat at the centre


@pytest.mark.parametrize("h", [0.2, 1.0, 2.5])
def test_kernel_normalised(h):
    val, err = integrate.quad(lambda r: 4 * math.pi * r * r * oracle.sph_kernel(r, h), 0, h, points=[h / 2],
                              epsabs=1e-13, epsrel=1e-12)
    assert val == pytest.approx(1.0, abs=1e-10)


@pytest.mark.parametrize("h,tol", [(2.0, 1e-3), (2.5, 5e-3), (3.0, 5e-3)])
def test_lattice_density(h, tol):
    g = np.arange(-6, 7, dtype=float)
    X, Y, Z = np.meshgrid(g, g, g, indexing="ij")
    pos = np.stack([X.ravel(), Y.ravel(), Z.ravel()], 1)
    centre = int(np.argmin(np.abs(pos).sum(1)))
    inner = np.flatnonzero(np.abs(pos).max(1) <= 2)         # support fully inside the lattice
    s = oracle.sph_sum(pos, np.full(len(pos), h), np.ones(len(pos)), tgt=inner)
    assert abs(s[list(inner).index(centre)] - 1.0) <= tol
    assert np.all(np.abs(s - 1.0) <= tol)                    # translation invariance of the interior
    assert np.ptp(s) < 1e-12


def test_two_particles_symmetrised():
    pos = np.array([[0.0, 0.0, 0.0], [0.5, 0.0, 0.0]])
    h = np.array([1.0, 2.0])
    q = np.array([3.0, 5.0])
    # W(0.5, 1) = 2/pi; W(0.5, 2): u = 1/4, w = 1 - 6/16 + 6/64 = 0.71875, sigma = 1/pi
    w01 = 0.5 * (2.0 / math.pi + 0.71875 / math.pi)
    s = oracle.sph_sum(pos, h, q)
    assert s[0] == pytest.approx(3.0 * 8.0 / math.pi + 5.0 * w01, rel=1e-14)
    assert s[1] == pytest.approx(5.0 * 1.0 / math.pi + 3.0 * w01, rel=1e-14)
    far = np.array([[0.0, 0.0, 0.0], [2.5, 0.0, 0.0]])        # beyond both supports
    s = oracle.sph_sum(far, h, q)
    assert s[0] == pytest.approx(3.0 * 8.0 / math.pi, rel=1e-15)
