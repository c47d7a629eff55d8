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


def _shell_average(k, p, kfund, n_shells):
    """Mean of p over shells [s, s+1) kfund of |k|, s = 1 .. n_shells - 1."""
    sh = np.floor(k.ravel() / kfund + 1e-9).astype(np.int64)
    kb, pb = [], []
    for s in range(1, n_shells):
        sel = sh == s
        kb.append(k.ravel()[sel].mean())
        pb.append(p.ravel()[sel].mean())
    return np.array(kb), np.array(pb)


def test_grf_cube_spectrum_and_rms_from_the_particles():
    """The cube's recipe measured from the particles alone (ng = 64).  Each
    particle k starts at lattice site q_k (cell centres, in generation order);
    its displacement psi = x - q is, by construction of a Zel'dovich field, a
    potential flow whose linear density contrast is delta = -div psi.  Taken
    from the particles by a spectral divergence: delta has rms 0.3 on the
    grid, psi has no curl, and the shell-averaged |delta_k|^2 falls as k^-2
    (log-log slope fitted between 2 k_f and k_Nyquist / 2).  The particles'
    own density (cloud-in-cell on the 64^3 grid, periodic wrap) follows the
    same spectrum at large scales: |delta_k|^2 within 10 % of the linear one
    in the first four shells and slope -2 within 0.1 up to 8 k_f, where the
    nonlinear and cloud-in-cell corrections are small."""
    ng = 64
    pos, m = synth.grf_cube(ng, seed=4)
    assert m.sum() == pytest.approx(1.0)
    idx = (np.arange(ng) + 0.5) / ng
    qx, qy, qz = np.meshgrid(idx, idx, idx, indexing="ij")
    psi = pos.reshape(ng, ng, ng, 3) - np.stack([qx, qy, qz], axis=-1)
    kf = 2 * math.pi * np.fft.fftfreq(ng, d=1.0 / ng)
    kr = 2 * math.pi * np.fft.rfftfreq(ng, d=1.0 / ng)
    K = [kf[:, None, None], kf[None, :, None], kr[None, None, :]]
    pk = [np.fft.rfftn(psi[..., a]) for a in range(3)]
    div = sum(1j * K[a] * pk[a] for a in range(3))
    delta_k = -div
    delta = np.fft.irfftn(delta_k, s=(ng, ng, ng), axes=(0, 1, 2))
    assert np.sqrt(np.mean(delta * delta)) == pytest.approx(0.3, rel=1e-4)
    curl = sum(np.abs(K[(a + 1) % 3] * pk[(a + 2) % 3] - K[(a + 2) % 3] * pk[(a + 1) % 3]) for a in range(3))
    assert curl.sum() <= 1e-10 * np.abs(div).sum()
    k = np.sqrt(K[0] ** 2 + K[1] ** 2 + K[2] ** 2)
    kfund = 2 * math.pi
    kb, pb = _shell_average(k, np.abs(delta_k) ** 2, kfund, ng // 2)
    sel = (kb >= 2 * kfund) & (kb <= math.pi * ng / 2)
    slope = np.polyfit(np.log(kb[sel]), np.log(pb[sel]), 1)[0]
    assert slope == pytest.approx(-2.0, abs=0.05)
    # cloud-in-cell density of the particles themselves
    x = pos * ng - 0.5
    i0 = np.floor(x).astype(np.int64)
    f = x - i0
    rho = np.zeros((ng, ng, ng))
    for dx in (0, 1):
        for dy in (0, 1):
            for dz in (0, 1):
                w = (f[:, 0] if dx else 1 - f[:, 0]) * (f[:, 1] if dy else 1 - f[:, 1]) * \
                    (f[:, 2] if dz else 1 - f[:, 2])
                np.add.at(rho, ((i0[:, 0] + dx) % ng, (i0[:, 1] + dy) % ng, (i0[:, 2] + dz) % ng), w)
    dc = np.fft.rfftn(rho / rho.mean() - 1.0)
    kc, pc = _shell_average(k, np.abs(dc) ** 2, kfund, 9)
    np.testing.assert_allclose(pc[:4] / pb[:4], 1.0, atol=0.1)
    assert np.polyfit(np.log(kc), np.log(pc), 1)[0] == pytest.approx(-2.0, abs=0.1)
