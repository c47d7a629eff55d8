"""Pins of the FP64 list force (oracle_list_force) and its quadrupole-form term.

* a cell entry whose moments are one particle's is that particle;
* a monopole at the centre of mass approximates a cell with an error that
  falls as (l/D)^2 (no dipole about the COM); adding the textbook quadrupole
  Q = 3S - tr(S) I makes it fall as (l/D)^3 -- this fixes the sign and the
  form of the quadrupole term;
* the quadrupole-form acceleration is minus the gradient of its potential;
* malformed lists are rejected.
"""
import numpy as np
import pytest

import oracle
from oracle import mlp as omlp


def _cluster(seed, n=40, size=0.1):
    rng = np.random.default_rng(seed)
    p = rng.uniform(-size / 2, size / 2, (n, 3)) * np.array([1.0, 0.6, 0.3])
    m = rng.uniform(0.5, 1.5, n)
    com = (m[:, None] * p).sum(0) / m.sum()
    r = p - com
    S = (m[:, None, None] * r[:, :, None] * r[:, None, :]).sum(0)
    return p, m, com, m.sum(), np.array([S[0, 0], S[1, 1], S[2, 2], S[0, 1], S[0, 2], S[1, 2]])


def test_cell_entry_equals_particle():
    rng = np.random.default_rng(1)
    pos = rng.normal(size=(10, 3))
    m = rng.uniform(0.5, 1.5, 10)
    # one group of all particles; list: particles 0..8 and particle 9 as a cell
    go = [0, 10]
    a_ref, p_ref = oracle.list_force(pos, m, go, [0, 10], np.arange(10), np.zeros((0, 3)), [], 0.01)
    a, p = oracle.list_force(pos, m, go, [0, 10], list(range(9)) + [10], pos[9:10], m[9:10], 0.01)
    # target 9 sees itself as a cell at distance 0: remove that row
    np.testing.assert_allclose(a[:9], a_ref[:9], rtol=1e-14)
    np.testing.assert_allclose(p[:9], p_ref[:9], rtol=1e-14)


def _monopole_and_quad_errors(D, direction, eps=0.0):
    p, m, com, M, S6 = _cluster(3)
    x = com + D * direction
    a_ex, _ = oracle.point_field(x[None], [0, len(m)], np.arange(len(m)), p, m, eps)
    # monopole through the list sum: one target particle of zero mass, one cell entry
    pos = np.vstack([x[None], p])
    mass = np.concatenate([[0.0], m])
    a_mono, _ = oracle.list_force(pos, mass, [0, 1, 1 + len(m)], [0, 1, 1], [1 + len(m)],
                                  com[None], [M], eps, tgt=[0])
    Q = omlp.exact_quadrupole(S6[None])
    a_mq, _ = oracle.list_force(pos, mass, [0, 1, 1 + len(m)], [0, 1, 1], [1 + len(m)],
                                com[None], [M], eps, tgt=[0], n_cellent=[1, 0], quad=Q)
    n = np.linalg.norm(a_ex)
    return np.linalg.norm(a_mono - a_ex) / n, np.linalg.norm(a_mq - a_ex) / n


@pytest.mark.parametrize("direction", [np.array([1.0, 0, 0]), np.array([0.3, -0.5, 0.81])])
def test_multipole_convergence_orders(direction):
    direction = direction / np.linalg.norm(direction)
    e1m, e1q = _monopole_and_quad_errors(1.0, direction)
    e2m, e2q = _monopole_and_quad_errors(2.0, direction)
    # monopole error ~ D^-2 relative; with the quadrupole ~ D^-3
    assert e1m / e2m == pytest.approx(4.0, rel=0.08)
    assert e1q / e2q == pytest.approx(8.0, rel=0.12)
    assert e1q < 0.2 * e1m


def test_quad_field_is_minus_gradient():
    rng = np.random.default_rng(5)
    c = np.zeros(3)
    q = rng.normal(size=6)
    q[2] = -q[0] - q[1]
    for eps in (0.0, 0.3):
        x = rng.normal(size=3) * 2
        a, _ = oracle.quad_field(x[None], c[None], q[None], eps)
        h = 1e-5
        grad = np.zeros(3)
        for k in range(3):
            e = np.zeros(3)
            e[k] = h
            _, pp = oracle.quad_field((x + e)[None], c[None], q[None], eps)
            _, pm = oracle.quad_field((x - e)[None], c[None], q[None], eps)
            grad[k] = (pp[0] - pm[0]) / (2 * h)
        np.testing.assert_allclose(a[0], -grad, rtol=1e-7, atol=1e-12)


def test_bad_lists_rejected():
    pos = np.zeros((2, 3))
    pos[1, 0] = 1
    with pytest.raises(ValueError):
        oracle.list_force(pos, [1, 1], [0, 2], [0, 1], [5], np.zeros((1, 3)), [1.0], 0.1)
    with pytest.raises(ValueError):   # particle entry where a cell tensor is promised
        oracle.list_force(pos, [1, 1], [0, 2], [0, 2], [0, 1], np.zeros((1, 3)), [1.0], 0.1,
                          n_cellent=[1], quad=np.zeros((1, 6)))


def test_quad_derivatives_are_derivatives_of_field():
    """J is the derivative of the field, H the derivative of J (central
    differences of independently coded functions), both symmetric."""
    rng = np.random.default_rng(12)
    q = rng.normal(size=6)
    c = np.zeros(3)
    hidx = [(0, 0, 0), (1, 1, 1), (2, 2, 2), (0, 0, 1), (0, 0, 2), (0, 1, 1), (1, 1, 2), (0, 2, 2), (1, 2, 2),
            (0, 1, 2)]
    for eps in (0.0, 0.2):
        x = rng.normal(size=3) * 2
        a, J, H, p = oracle.quad_derivs(x[None], c[None], q[None], eps)
        a2, p2 = oracle.quad_field(x[None], c[None], q[None], eps)
        np.testing.assert_allclose(a, a2, rtol=1e-13)
        np.testing.assert_allclose(p, p2, rtol=1e-13)
        h = 1e-5
        Jfd = np.zeros((3, 3))
        Hfd = np.zeros((3, 3, 3))
        for k in range(3):
            e = np.zeros(3)
            e[k] = h
            ap, _ = oracle.quad_field((x + e)[None], c[None], q[None], eps)
            am, _ = oracle.quad_field((x - e)[None], c[None], q[None], eps)
            Jfd[:, k] = (ap[0] - am[0]) / (2 * h)
            _, Jp, _, _ = oracle.quad_derivs((x + e)[None], c[None], q[None], eps)
            _, Jm, _, _ = oracle.quad_derivs((x - e)[None], c[None], q[None], eps)
            dJ = (Jp[0] - Jm[0]) / (2 * h)
            full = np.array([[dJ[0], dJ[3], dJ[4]], [dJ[3], dJ[1], dJ[5]], [dJ[4], dJ[5], dJ[2]]])
            Hfd[:, :, k] = full
        J6 = np.array([Jfd[0, 0], Jfd[1, 1], Jfd[2, 2], Jfd[0, 1], Jfd[0, 2], Jfd[1, 2]])
        np.testing.assert_allclose(J[0], J6, rtol=1e-6, atol=1e-9 * np.abs(J6).max())
        H10 = np.array([Hfd[i, j, k] for i, j, k in hidx])
        np.testing.assert_allclose(H[0], H10, rtol=1e-5, atol=1e-8 * np.abs(H10).max())
        # full symmetry of the finite-difference third derivative
        np.testing.assert_allclose(Hfd, Hfd.transpose(0, 2, 1), atol=1e-5 * np.abs(Hfd).max())
        np.testing.assert_allclose(Hfd, Hfd.transpose(2, 1, 0), atol=1e-5 * np.abs(Hfd).max())


def _expanded_vs_exact(spread):
    # one group of 10 targets near the origin, cells far away carrying tensors
    rng = np.random.default_rng(13)
    tg = rng.uniform(-spread, spread, (10, 3))
    com = np.array([[3.0, 0.5, -0.2], [-2.0, 2.5, 1.0]])
    pos = np.vstack([tg])
    m = np.full(10, 1e-3)
    q = rng.normal(size=(2, 6)) * 0.1
    args = (pos, m, [0, 10], [0, 12], [10, 11] + list(range(10)), com, [1.0, 2.0], 0.01)
    a_ex, p_ex = oracle.list_force(*args, n_cellent=[2], quad=q)
    a_lx, p_lx = oracle.list_force(*args, n_cellent=[2], quad=q, expanded=True)
    a_mo, p_mo = oracle.list_force(*args)
    return (np.abs(a_lx - a_ex).max(), np.abs(p_lx - p_ex).max(),
            np.abs(a_ex - a_mo).max())


def test_local_expansion_is_third_order():
    # second-order expansion: the error falls as spread^3 (the potential as spread^3 too)
    d1, p1, corr1 = _expanded_vs_exact(0.2)
    d2, p2, corr2 = _expanded_vs_exact(0.1)
    assert d1 < 0.01 * corr1
    assert d1 / d2 == pytest.approx(8.0, rel=0.15)
    assert p1 / p2 == pytest.approx(8.0, rel=0.15)


def test_local_expansion_zero_tensor_is_monopole():
    rng = np.random.default_rng(14)
    pos = rng.normal(size=(20, 3))
    m = rng.uniform(0.5, 1.5, 20)
    args = (pos, m, [0, 10, 20], [0, 11, 22], [20] + list(range(10)) + [20] + list(range(10, 20)),
            np.array([[5.0, 5.0, 5.0]]), [3.0], 0.05)
    a0, p0 = oracle.list_force(*args)
    a1, p1 = oracle.list_force(*args, n_cellent=[1, 1], quad=np.zeros((2, 6)), expanded=True)
    np.testing.assert_array_equal(a0, a1)
    np.testing.assert_array_equal(p0, p1)


@pytest.mark.parametrize("group_mode", [0, 1])
def test_expansion_within_truncation_bound_on_real_groups(group_mode):
    """The second-order local expansion about each group's box centre (the
    form the device applies) against the per-particle quadrupole form (the
    definition), both in the FP64 oracle, on real groups of up to 128
    particles at opening angle 0.9 (Plummer 2^16, textbook tensors
    3 S - tr(S) I): per target the difference stays within the derived
    truncation bound (tests/learned_helpers.py), and the expansion keeps most
    of the quadrupole term (its median error is under half the term's median
    size).  The bound is rigorous but loose (about 100x the measured error at
    these group sizes), so the GPU parity tests against the per-particle form
    also compare the device's median deviation with the truncation measured
    here."""
    import synth
    import paper_1206_1199_amd as otoo
    from oracle import mlp as omlp
    from learned_helpers import group_geometry, nuclear_norm6, pair_index, sub_lists, target_bounds
    eps = 0.005
    pos, m = synth.plummer(1 << 16, seed=21)
    tree = otoo.Tree(pos, m, n_crit=16)
    lists = tree.walk(theta=0.9, g_max=128, group_mode=group_mode)
    _, pos32, mass32, cm = tree.export(12)
    p64, m64 = pos32.astype(np.float64), mass32.astype(np.float64)
    n = len(m64)
    rng = np.random.default_rng(5)
    groups = np.sort(rng.choice(lists.n_groups, 64, replace=False))
    tgt = np.concatenate([np.arange(lists.group_off[g], lists.group_off[g + 1])[:8] for g in groups])
    sub = sub_lists(lists, groups)
    _, c_all = pair_index(lists, n)
    cells = c_all[sub["pairs"]]
    Q = omlp.exact_quadrupole(cm[cells, 5:11].astype(np.float64))
    args = (p64, m64, sub["group_off"], sub["list_off"], sub["list_idx"], cm[:, :3].astype(np.float64),
            cm[:, 3].astype(np.float64), eps)
    a_pp, p_pp = oracle.list_force(*args, tgt=tgt, n_cellent=sub["n_cellent"], quad=Q)
    a_ex, p_ex = oracle.list_force(*args, tgt=tgt, n_cellent=sub["n_cellent"], quad=Q, expanded=True)
    a_mo, _ = oracle.list_force(*args, tgt=tgt)
    centre, _ = group_geometry(p64, lists.group_off)
    ba, bp = target_bounds(p64, lists.group_off, centre, tgt, sub, cm[:, :3].astype(np.float64), nuclear_norm6(Q),
                           n, eps)
    da = np.linalg.norm(a_ex - a_pp, axis=1)
    dp = np.abs(p_ex - p_pp)
    an = np.linalg.norm(a_pp, axis=1)
    corr = np.linalg.norm(a_pp - a_mo, axis=1)
    print(f"group mode {group_mode}: expansion error median {np.median(da / an):.2e} max {np.max(da / an):.2e}; "
          f"bound median {np.median(ba / an):.2e} max {np.max(ba / an):.2e}; quadrupole term median "
          f"{np.median(corr / an):.2e} of the force", flush=True)
    assert np.all(da <= ba + 1e-12 * an)
    assert np.all(dp <= bp + 1e-12 * np.abs(p_pp))
    assert np.median(da) < 0.5 * np.median(corr)


def test_cells_after_the_tensor_range_are_monopoles():
    """Tensors cover the first n_cellent[g] entries; a cell entry after them
    (a far cell behind a list's near cells) acts as a monopole only: the same
    sums as giving that cell a zero tensor."""
    rng = np.random.default_rng(31)
    pos = rng.normal(size=(3, 3))
    mass = np.array([1.0, 2.0, 0.5])
    com = rng.normal(size=(2, 3)) * 4.0
    cmass = np.array([3.0, 1.5])
    q = rng.normal(size=(1, 6))
    args = (pos, mass, [0, 3], [0, 5], [3, 4, 0, 1, 2], com, cmass, 0.05)
    for expanded in (False, True):
        a1, p1 = oracle.list_force(*args, n_cellent=[1], quad=q, expanded=expanded)
        a2, p2 = oracle.list_force(*args, n_cellent=[2], quad=np.concatenate([q, np.zeros((1, 6))]),
                                   expanded=expanded)
        np.testing.assert_allclose(a1, a2, rtol=1e-14, atol=0)
        np.testing.assert_allclose(p1, p2, rtol=1e-14, atol=0)
