"""Seeded synthetic particle distributions (positions and masses only).

This module is shared by the FP64 oracle (``oracle/``), the tests and the
product path.  It holds no force, tree or walk arithmetic: it only draws
particles.  Every generator takes an explicit seed and uses NumPy's PCG64 bit
generator, so both sides see bit-identical inputs.

Distributions (all with G = 1):

* ``plummer``        Plummer sphere, the astrophysical test model named in the
                     gravity performance section (Sec. 4.1) of the paper.
* ``uniform_sphere`` uniform-density sphere r <= 1, M = 1 (Sec. 3.4 and 4.1).
* ``polytrope_pair`` two n = 1.5 polytropes, a gravity-only stand-in for the
                     white-dwarf pair of Sec. 5 (the initial models used there
                     are not available).
* ``grf_cube``       isolated unit cube of N = ng^3 particles displaced from a
                     lattice by a Gaussian random field with P(k) ~ k^-2.
"""
from __future__ import annotations

import functools
import math

import numpy as np


def rng_for(seed: int) -> np.random.Generator:
    """The one bit generator every input draw goes through."""
    return np.random.Generator(np.random.PCG64(int(seed)))


def _isotropic(rng: np.random.Generator, n: int) -> np.ndarray:
    """Unit vectors uniform on the sphere (Archimedes: cos(theta) ~ U(-1, 1))."""
    mu = rng.uniform(-1.0, 1.0, n)
    phi = rng.uniform(0.0, 2.0 * math.pi, n)
    s = np.sqrt(np.maximum(0.0, 1.0 - mu * mu))
    return np.stack([s * np.cos(phi), s * np.sin(phi), mu], axis=1)


def plummer(n: int, seed: int, a: float = 1.0, mass: float = 1.0,
            x_max: float = 0.999, recentre: bool = True):
    """Plummer sphere of ``n`` equal-mass particles.

    The enclosed-mass fraction of a Plummer sphere is X(r) = r^3 (r^2 + a^2)^-3/2
    (with r in units of a).  A radius is drawn by inverting it for
    X ~ U(0, x_max): r = a (X^-2/3 - 1)^-1/2; ``x_max`` < 1 truncates the
    infinite tail at R_cut = a (x_max^-2/3 - 1)^-1/2 (38.7 a for 0.999).
    Directions are isotropic.  With ``recentre`` the sample's centre of mass is
    moved to the origin.

    Returns (pos[n,3] float64, m[n] float64).
    """
    rng = rng_for(seed)
    x = rng.uniform(0.0, x_max, n)
    r = a / np.sqrt(np.power(x, -2.0 / 3.0) - 1.0)
    pos = r[:, None] * _isotropic(rng, n)
    if recentre:
        pos -= pos.mean(axis=0)
    m = np.full(n, mass / n)
    return pos, m


def uniform_sphere(n: int, seed: int, radius: float = 1.0, mass: float = 1.0):
    """Uniform-density sphere: r = R u^(1/3), u ~ U(0, 1), isotropic."""
    rng = rng_for(seed)
    r = radius * np.cbrt(rng.uniform(0.0, 1.0, n))
    pos = r[:, None] * _isotropic(rng, n)
    return pos, np.full(n, mass / n)


@functools.lru_cache(maxsize=4)
def lane_emden(n_index: float = 1.5, h: float = 1e-4):
    """Solve the Lane-Emden equation theta'' + (2/xi) theta' + theta^n = 0 with RK4.

    Starts at a small xi from the series theta = 1 - xi^2/6 + n xi^4/120 and
    stops at the first zero xi_1 (located by linear interpolation of the last
    step).  Returns (xi, theta, dtheta, xi_1, dtheta_1) with the arrays
    truncated at the last grid point inside the star.
    """
    nn = float(n_index)

    def rhs(xi, th, dth):
        return dth, -(max(th, 0.0) ** nn) - 2.0 * dth / xi

    xi = 1e-6
    th = 1.0 - xi * xi / 6.0 + nn * xi ** 4 / 120.0
    dth = -xi / 3.0 + nn * xi ** 3 / 30.0
    xs, ths, dths = [0.0, xi], [1.0, th], [0.0, dth]
    while True:
        k1a, k1b = rhs(xi, th, dth)
        k2a, k2b = rhs(xi + h / 2, th + h / 2 * k1a, dth + h / 2 * k1b)
        k3a, k3b = rhs(xi + h / 2, th + h / 2 * k2a, dth + h / 2 * k2b)
        k4a, k4b = rhs(xi + h, th + h * k3a, dth + h * k3b)
        th_n = th + h / 6 * (k1a + 2 * k2a + 2 * k3a + k4a)
        dth_n = dth + h / 6 * (k1b + 2 * k2b + 2 * k3b + k4b)
        if th_n <= 0.0:
            frac = th / (th - th_n)
            xi1 = xi + frac * h
            dth1 = dth + frac * (dth_n - dth)
            return (np.array(xs), np.array(ths), np.array(dths), xi1, dth1)
        xi += h
        th, dth = th_n, dth_n
        xs.append(xi)
        ths.append(th)
        dths.append(dth)


def polytrope(n: int, rng: np.random.Generator, radius: float, mass: float,
              n_index: float = 1.5):
    """``n`` equal-mass particles sampling an n-index polytrope of given R and M.

    The enclosed mass at xi is proportional to -xi^2 theta'(xi); a radius is
    drawn by inverting the normalised enclosed-mass profile with linear
    interpolation on the RK4 grid.
    """
    xs, _, dths, xi1, dth1 = lane_emden(n_index)
    menc = np.append(-xs * xs * dths, -xi1 * xi1 * dth1)
    xg = np.append(xs, xi1)
    menc = menc / menc[-1]
    u = rng.uniform(0.0, 1.0, n)
    xi = np.interp(u, menc, xg)
    pos = (radius * xi / xi1)[:, None] * _isotropic(rng, n)
    return pos, np.full(n, mass / n)


def polytrope_pair(n_each: int, seed: int, m_a: float = 0.6, r_a: float = 0.02,
                   m_b: float = 0.9, r_b: float = 0.012, sep: float = 0.05):
    """Two n = 1.5 polytropes, ``n_each`` particles each, centres ``sep`` apart on x.

    Star A (m_a, r_a) sits at x = -sep m_b/(m_a+m_b) and star B at
    x = +sep m_a/(m_a+m_b), so the pair's analytic centre of mass is the
    origin.  Particles within a star have equal mass (m_a/n_each or
    m_b/n_each).

    Returns (pos[2 n_each, 3], m[2 n_each], star[2 n_each] int8, centres[2,3]).
    """
    rng = rng_for(seed)
    ca = np.array([-sep * m_b / (m_a + m_b), 0.0, 0.0])
    cb = np.array([sep * m_a / (m_a + m_b), 0.0, 0.0])
    pa, ma = polytrope(n_each, rng, r_a, m_a)
    pb, mb = polytrope(n_each, rng, r_b, m_b)
    pos = np.concatenate([pa + ca, pb + cb])
    m = np.concatenate([ma, mb])
    star = np.concatenate([np.zeros(n_each, np.int8), np.ones(n_each, np.int8)])
    return pos, m, star, np.stack([ca, cb])


def grf_cube(ng: int, seed: int, rms: float = 0.3, slope: float = -2.0,
             box: float = 1.0, mass: float = 1.0):
    """Isolated cube of ng^3 particles perturbed by a Gaussian random field.

    A white-noise grid is filtered in Fourier space by sqrt(P(k)) with
    P(k) ~ k^slope for 0 < |k| <= k_Nyquist (k = 0 removed) and rescaled so
    the density contrast delta has the requested rms on the grid.  Particles
    start at cell centres q and move by the Zel'dovich displacement
    psi_k = i k delta_k / k^2 (so that delta = -div psi).  The boundaries are
    open: the cube is not periodic for the force, only the field is.  With
    rms = 0 the result is the unperturbed lattice.

    Returns (pos[ng^3, 3] float64, m[ng^3] float64).
    """
    n = ng ** 3
    idx = (np.arange(ng, dtype=np.float64) + 0.5) * (box / ng)
    qx, qy, qz = np.meshgrid(idx, idx, idx, indexing="ij")
    if rms == 0.0:
        pos = np.stack([qx.ravel(), qy.ravel(), qz.ravel()], axis=1)
        return pos, np.full(n, mass / n)
    rng = rng_for(seed)
    white = rng.standard_normal((ng, ng, ng))
    wk = np.fft.rfftn(white)
    kf = 2.0 * math.pi * np.fft.fftfreq(ng, d=box / ng)
    kr = 2.0 * math.pi * np.fft.rfftfreq(ng, d=box / ng)
    kx = kf[:, None, None]
    ky = kf[None, :, None]
    kz = kr[None, None, :]
    k2 = kx * kx + ky * ky + kz * kz
    knyq = math.pi * ng / box
    with np.errstate(divide="ignore", invalid="ignore"):
        amp = np.where((k2 > 0) & (k2 <= knyq * knyq), np.power(k2, slope / 4.0), 0.0)
    dk = wk * amp
    del wk
    delta = np.fft.irfftn(dk, s=(ng, ng, ng), axes=(0, 1, 2))
    scale = rms / np.sqrt(np.mean(delta * delta))
    del delta
    dk *= scale
    with np.errstate(divide="ignore", invalid="ignore"):
        inv_k2 = np.where(k2 > 0, 1.0 / k2, 0.0)
    pos = np.empty((n, 3))
    for ax, (kk, q) in enumerate(((kx, qx), (ky, qy), (kz, qz))):
        psi = np.fft.irfftn(1j * kk * dk * inv_k2, s=(ng, ng, ng), axes=(0, 1, 2))
        pos[:, ax] = (q + psi).ravel()
        del psi
    return pos, np.full(n, mass / n)


def knn_radius(pos: np.ndarray, k: int = 32) -> np.ndarray:
    """Distance from each point to its k-th nearest other point: the
    neighbour radius h of an SPH particle with about k neighbours."""
    from scipy.spatial import cKDTree
    d, _ = cKDTree(pos).query(pos, k=k + 1, workers=-1)
    return d[:, -1].astype(np.float64)


def sample_idx(n: int, k: int, seed: int) -> np.ndarray:
    """``k`` distinct indices of [0, n) drawn without replacement, ascending."""
    rng = rng_for(seed)
    k = min(k, n)
    return np.sort(rng.choice(n, size=k, replace=False)).astype(np.int64)
