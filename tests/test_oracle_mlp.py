"""Pins of the FP64 network oracle (oracle/mlp.py).

* tanh-GELU against the exact erf form (a textbook routine) and known limits;
* the hand-written backward against central finite differences of the
  forward and loss;
* the quadrupole basis against the C oracle's quadrupole field;
* the loss reaches zero gradient at the per-pair least-squares tensor and the
  exact quadrupole Q = 3S - tr(S) I explains the monopole error far away;
* the first Adam step moves every parameter by lr against its gradient sign.
"""
import math

import numpy as np
import pytest
from scipy import special

import oracle
from oracle import mlp as omlp


def test_gelu_values():
    z = np.linspace(-6, 6, 241)
    exact = 0.5 * z * (1 + special.erf(z / math.sqrt(2)))
    assert np.max(np.abs(omlp.gelu(z) - exact)) < 1e-3
    assert omlp.gelu(np.array([0.0]))[0] == 0.0
    assert omlp.gelu(np.array([20.0]))[0] == pytest.approx(20.0, rel=1e-12)
    assert abs(omlp.gelu(np.array([-20.0]))[0]) < 1e-12
    h = 1e-6
    zz = np.array([-2.0, -0.3, 0.0, 0.7, 3.0])
    fd = (omlp.gelu(zz + h) - omlp.gelu(zz - h)) / (2 * h)
    np.testing.assert_allclose(omlp.gelu_grad(zz), fd, rtol=1e-8, atol=1e-10)


def _batch(seed, P=40):
    rng = np.random.default_rng(seed)
    d = rng.normal(size=(P, 3))
    d *= (3.0 / np.linalg.norm(d, axis=1))[:, None]
    l_c = rng.uniform(0.5, 1.0, P)
    M_c = rng.uniform(0.5, 2.0, P)
    S = rng.normal(size=(P, 6)) * 0.05
    u = omlp.features(d, l_c, 0.01, rng.uniform(0.1, 0.5, P), S, M_c)
    dvec = rng.normal(size=(P, 3)) * 2.5
    t = rng.normal(size=(P, 3)) * 1e-3
    return u, dvec, M_c, l_c, t


def test_backward_matches_finite_differences():
    p = omlp.init_params(0)
    for k in p:
        p[k] = p[k] + np.random.default_rng(1).normal(size=p[k].shape) * 0.05
    u, dvec, M_c, l_c, t = _batch(2)
    w = np.random.default_rng(2).uniform(0.2, 3.0, len(u))
    L, g, _ = omlp.loss_and_grad(p, u, dvec, M_c, l_c, t, 0.01, w)
    assert L == pytest.approx(omlp.loss(p, u, dvec, M_c, l_c, t, 0.01, w), rel=1e-14)
    rng = np.random.default_rng(3)
    for k in p:
        flat = p[k].reshape(-1)
        for j in rng.choice(flat.size, size=min(6, flat.size), replace=False):
            h = 1e-6 * max(1.0, abs(flat[j]))
            q = {kk: vv.copy() for kk, vv in p.items()}
            q[k].reshape(-1)[j] += h
            lp = omlp.loss(q, u, dvec, M_c, l_c, t, 0.01, w)
            q[k].reshape(-1)[j] -= 2 * h
            lm = omlp.loss(q, u, dvec, M_c, l_c, t, 0.01, w)
            fd = (lp - lm) / (2 * h)
            assert g[k].reshape(-1)[j] == pytest.approx(fd, rel=1e-6, abs=1e-9 * abs(L) + 1e-14)


def test_quad_basis_matches_c_oracle():
    rng = np.random.default_rng(4)
    d = rng.normal(size=(20, 3))
    q = rng.normal(size=(20, 6))
    a_c, _ = oracle.quad_field(d, np.zeros((20, 3)), q, 0.2)
    a_np = np.einsum("pkj,pj->pk", omlp.quad_accel_basis(d, 0.2), q)
    np.testing.assert_allclose(a_np, a_c, rtol=1e-12, atol=1e-14)


def test_traceless_projection():
    o = np.random.default_rng(6).normal(size=(10, 6))
    q = omlp.traceless(o)
    np.testing.assert_allclose(q[:, 0] + q[:, 1] + q[:, 2], 0, atol=1e-14)
    np.testing.assert_allclose(omlp.traceless(q), q, atol=1e-15)
    np.testing.assert_array_equal(q[:, 3:], o[:, 3:])


def test_exact_quadrupole_explains_far_field():
    # a distant cluster: a_exact - a_mono is the quadrupole field of
    # Q = 3S - tr(S) I to relative O(l/D)
    rng = np.random.default_rng(8)
    p = rng.uniform(-0.05, 0.05, (30, 3)) * np.array([1.0, 0.5, 0.2])
    m = rng.uniform(0.5, 1.5, 30)
    com = (m[:, None] * p).sum(0) / m.sum()
    r = p - com
    S = (m[:, None, None] * r[:, :, None] * r[:, None, :]).sum(0)
    S6 = np.array([[S[0, 0], S[1, 1], S[2, 2], S[0, 1], S[0, 2], S[1, 2]]])
    for D in (1.0, 4.0):
        x = com + D * np.array([0.6, 0.64, 0.48])
        a_ex, _ = oracle.point_field(x[None], [0, 30], np.arange(30), p, m, 0.0)
        a_mono, _ = oracle.point_field(x[None], [0, 1], [0], com[None], [m.sum()], 0.0)
        a_q = np.einsum("pkj,pj->pk", omlp.quad_accel_basis((x - com)[None], 0.0),
                        omlp.exact_quadrupole(S6))
        err = np.linalg.norm(a_ex - a_mono - a_q) / np.linalg.norm(a_ex - a_mono)
        assert err < 0.06 / D


def test_least_squares_tensor_zero_gradient():
    # the per-sample loss is quadratic in Qt; at its minimiser the gradient
    # with respect to the network output vanishes (checked through do).
    rng = np.random.default_rng(9)
    P = 12
    dvec = rng.normal(size=(P, 3)) * 3
    B = omlp.quad_accel_basis(dvec, 0.01)
    t = rng.normal(size=(P, 3)) * 1e-3
    # all samples share one pair: solve the 6x6 normal equations
    w = ((dvec ** 2).sum(1)) ** 2
    A = np.einsum("p,pkj,pki->ji", w, B, B)
    b = np.einsum("p,pkj,pk->j", w, B, t)
    # restrict to traceless tensors: parametrise by (xx, yy, xy, xz, yz)
    T = np.zeros((6, 5))
    T[0, 0] = T[1, 1] = 1
    T[2, 0] = T[2, 1] = -1
    T[3, 2] = T[4, 3] = T[5, 4] = 1
    q5 = np.linalg.solve(T.T @ A @ T, T.T @ b)
    q = T @ q5
    r = np.einsum("pkj,j->pk", B, q) - t
    grad_q = np.einsum("p,pkj,pk->j", w, B, r)
    np.testing.assert_allclose(T.T @ grad_q, 0, atol=1e-10 * np.abs(T.T @ b).max())


def test_adam_first_step():
    p = {"w": np.array([1.0, -2.0, 3.0])}
    g = {"w": np.array([0.5, -1e-3, 2.0])}
    z = {"w": np.zeros(3)}
    p1, m1, v1 = omlp.adam_step(p, g, z, z, step=1, lr=0.01, eps=0.0)
    np.testing.assert_allclose(p1["w"], p["w"] - 0.01 * np.sign(g["w"]), rtol=1e-14)


def test_bf16_rounding_ties_to_even():
    v = np.array([1.0, 1 + 2 ** -8, 1 + 3 * 2 ** -8, 1 + 2 ** -8 + 2 ** -20, -(1 + 3 * 2 ** -8), 0.0, 3.0e38,
                  1.0 / 3.0])
    # 3e38 is 0x7F61B1E6 in FP32 -> 0x7F62 = (1 + 98/128) 2^127; 1/3 -> 0x3EAB = (1 + 43/128) / 4
    ref = np.array([1.0, 1.0, 1 + 2 ** -6, 1 + 2 ** -7, -(1 + 2 ** -6), 0.0, (1 + 98 / 128) * 2.0 ** 127,
                    (1 + 43 / 128) / 4])
    got = omlp.to_bf16(v)
    np.testing.assert_array_equal(got, ref)
    # every BF16 value is exact in 8 significant bits
    m, e = np.frexp(got[got != 0])
    np.testing.assert_array_equal(m * 256, np.round(m * 256))


def test_flat_parameter_layout_round_trip():
    p = omlp.init_params(3)
    v = omlp.params_to_flat(p)
    assert v.size == 6662
    q = omlp.flat_to_params(v)
    for k in p:
        np.testing.assert_array_equal(p[k], q[k])


def test_expanded_basis_matches_c_expansion():
    """B(D, delta) q is what the C oracle's expanded list force adds to the monopole."""
    rng = np.random.default_rng(31)
    tg = rng.uniform(-0.2, 0.2, (8, 3))
    com = np.array([[2.0, -1.0, 0.7]])
    q = rng.normal(size=(1, 6))
    args = (tg, np.full(8, 1e-3), [0, 8], [0, 9], [8] + list(range(8)), com, [1.5], 0.02)
    a_x, _ = oracle.list_force(*args, n_cellent=[1], quad=q, expanded=True)
    a_m, _ = oracle.list_force(*args)
    cg = 0.5 * (tg.min(0) + tg.max(0))
    B = omlp.expanded_basis(np.repeat((cg - com), 8, axis=0), tg - cg, 0.02)
    np.testing.assert_allclose(np.einsum("pkj,j->pk", B, q[0]), a_x - a_m, rtol=1e-10,
                               atol=1e-12 * np.abs(a_x - a_m).max())


def test_basis_backward_matches_finite_differences():
    p = omlp.init_params(5)
    rng = np.random.default_rng(6)
    P = 24
    u = rng.normal(size=(P, 32)) * 0.5
    B = rng.normal(size=(P, 3, 6))
    scale = rng.uniform(0.5, 2.0, P)
    t = rng.normal(size=(P, 3)) * 0.1
    w = rng.uniform(0.1, 1.0, P)
    L, g = omlp.loss_and_grad_basis(p, u, B, scale, t, w)
    def lossf(pp):
        o, _ = omlp.forward(pp, u)
        r = np.einsum("pkj,pj->pk", B, omlp.traceless(o) * scale[:, None]) - t
        return float(np.mean(w * (r * r).sum(1)))
    assert L == pytest.approx(lossf(p), rel=1e-14)
    for k in p:
        flat = p[k].reshape(-1)
        for j in rng.choice(flat.size, size=min(5, flat.size), replace=False):
            h = 1e-6
            q = {kk: vv.copy() for kk, vv in p.items()}
            q[k].reshape(-1)[j] += h
            lp = lossf(q)
            q[k].reshape(-1)[j] -= 2 * h
            lm = lossf(q)
            assert g[k].reshape(-1)[j] == pytest.approx((lp - lm) / (2 * h), rel=1e-6, abs=1e-10 * abs(L) + 1e-14)


def test_zero_layers_give_the_textbook_quadrupole():
    """With every weight and bias zero the outputs are the skip term alone, and
    M l^2 P(o) is the textbook quadrupole 3 S - tr(S) I of the cell (closed
    form), independent of the other features; a gate above every l/n does the
    same for any weights."""
    rng = np.random.default_rng(5)
    P = 30
    S = rng.normal(size=(P, 6))
    S[:, :3] = np.abs(S[:, :3]) + 1.0
    M = rng.uniform(0.5, 2.0, P)
    l = rng.uniform(0.1, 1.0, P)
    u = omlp.features(rng.normal(size=(P, 3)) * 5, l, 0.01, rng.uniform(0, 1, P), S, M)
    zero = {k: np.zeros_like(v) for k, v in omlp.init_params(0).items()}
    o, _ = omlp.forward(zero, u)
    q = omlp.traceless(o) * (M * l * l)[:, None]
    np.testing.assert_allclose(q, omlp.exact_quadrupole(S), rtol=1e-12, atol=1e-12)
    p = omlp.init_params(3)
    og = omlp.gated_outputs(p, u, gate=np.inf)
    np.testing.assert_allclose(omlp.traceless(og) * (M * l * l)[:, None], omlp.exact_quadrupole(S), rtol=1e-12,
                               atol=1e-12)
    # gate 0 leaves every pair to the layers
    np.testing.assert_array_equal(omlp.gated_outputs(p, u, gate=0.0), omlp.forward(p, u)[0])


def test_sample_weights_by_hand():
    """Two kept samples with |t|^2/|a|^2 = 1 and 3 give W = 2 / 4 = 1/2, so
    w = 1/2 / |a|^2; a sample the gate drops gets the same form of weight but
    leaves W unchanged; the kept samples' mean of w |t|^2 is then 1, and a
    target at rest keeps a finite weight."""
    a = np.array([[1.0, 0.0, 0.0], [0.0, 2.0, 0.0], [0.0, 0.0, 3.0], [0.0, 0.0, 0.0]])
    t = np.array([[1.0, 0.0, 0.0], [0.0, 0.0, 2.0 * np.sqrt(3.0)], [5.0, 0.0, 0.0], [1.0, 0.0, 0.0]])
    kept = np.array([True, True, False, False])
    w = omlp.sample_weights(a, t, kept)
    np.testing.assert_allclose(w[:3], [0.5, 0.125, 0.5 / 9.0], rtol=1e-15)
    assert w[3] == pytest.approx(0.5e300)
    assert np.mean((w * (t * t).sum(axis=1))[kept]) == pytest.approx(1.0, rel=1e-15)
    assert np.all(omlp.sample_weights(a[:2], np.zeros((2, 3)), kept[:2]) == 1.0 / np.array([1.0, 4.0]))
