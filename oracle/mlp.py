"""FP64 oracle of the learned monopole correction -- TEST INFRASTRUCTURE ONLY.

Not from the paper: the paper evaluates accepted cells as monopoles only and
names higher orders (up to the quadrupole, p = 3 in its counting) without
using them (Sec. 2).  The learned part predicts, for every (group g, accepted
cell c) pair, an effective symmetric traceless tensor Qt_gc whose
quadrupole-form field (same form as ``oracle_list_force``'s cell tensor) is
added to the cell's monopole.

Network:   u (12 features, zero-padded to 32)
           h1 = gelu(u W1 + b1)        W1 [32, 64]
           h2 = gelu(h1 W2 + b2)       W2 [64, 64]
           o  = h2 W3 + b3 + 3 s       W3 [64, 6]; s = u[6:12], the normalised S
           Qt = M_c l_c^2 * P(o)       P removes the trace: o_aa -= tr(o)/3
The fixed skip term 3 s makes M_c l_c^2 P(3 s) = 3 S - tr(S) I, the textbook
quadrupole: the layers learn the correction to it, and zero weights give
the quadrupole exactly.  With a gate tau > 0 the layers run only for pairs
whose feature l_c/n is at least tau; other pairs keep o = 3 s.  Both the
skip and the gate read the BF16-rounded features the network sees.
gelu is the tanh form of Hendrycks & Gimpel (2016):
           gelu(z) = z/2 (1 + tanh(sqrt(2/pi) (z + 0.044715 z^3))).

Features of a pair, with d = COM_c - centre_g (centre of group g's bounding
box) and n = |d|:
           d/n (3), l_c/n, eps/n, h_g/n (h_g = half-diagonal of the group
           box), S_c / (M_c l_c^2) as (xx, yy, zz, xy, xz, yz).

Loss over samples (g, c, target particle x_i of g):
           r = a_mono + a_Qt - a_exact,   L = mean(w |r|^2)
a_exact is the cell's exact softened direct sum at x_i.  Only the
Qt-dependent part of r needs the network, so a sample carries
t = a_exact - a_mono.  The weight (``sample_weights``; not in the paper) is
           w = W / |a_i|^2,  W = K / sum_kept |t|^2 / |a_i|^2
with a_i the total force on the target from the same walk and K the number
of samples the gate keeps, so that the loss follows the per-particle
relative force error (the measure the method is judged by) and the kept
samples' zero-correction loss, mean(w |t|^2), is 1.

The device applies each pair's tensor through a second-order local expansion
about the group's box centre c_g; ``expanded_basis`` gives that linear map
(from the C oracle's field derivatives) and ``loss_and_grad_basis`` the loss
with it.  ``to_bf16`` rounds to BF16 (round to nearest, ties to even) so the
oracle can run the network at the device's rounded weights and inputs.

Backward is written out by hand (reverse mode), and is checked against
central finite differences of ``forward``.
"""
from __future__ import annotations

import math

import numpy as np

N_IN = 32
N_FEAT = 12
N_H = 64
N_OUT = 6
GELU_C = math.sqrt(2.0 / math.pi)


def gelu(z):
    return 0.5 * z * (1.0 + np.tanh(GELU_C * (z + 0.044715 * z ** 3)))


def gelu_grad(z):
    inner = GELU_C * (z + 0.044715 * z ** 3)
    t = np.tanh(inner)
    dinner = GELU_C * (1.0 + 3.0 * 0.044715 * z * z)
    return 0.5 * (1.0 + t) + 0.5 * z * (1.0 - t * t) * dinner


def init_params(seed: int):
    """He-style uniform initialisation from a PCG64 stream (weights only)."""
    rng = np.random.Generator(np.random.PCG64(seed))

    def lin(n_in, n_out):
        lim = math.sqrt(6.0 / n_in)
        return rng.uniform(-lim, lim, (n_in, n_out)), np.zeros(n_out)

    W1, b1 = lin(N_IN, N_H)
    W2, b2 = lin(N_H, N_H)
    W3, b3 = lin(N_H, N_OUT)
    W3 *= 0.1
    return {"W1": W1, "b1": b1, "W2": W2, "b2": b2, "W3": W3, "b3": b3}


def features(d, l_c, eps, h_g, S_c, M_c):
    """Per-pair features (rows), zero-padded to N_IN columns.

    d[P,3] = COM_c - centre_g, l_c[P], h_g[P], S_c[P,6] (xx,yy,zz,xy,xz,yz),
    M_c[P]; eps scalar.
    """
    d = np.asarray(d, dtype=np.float64)
    n = np.sqrt((d * d).sum(axis=1))
    u = np.zeros((len(d), N_IN))
    u[:, 0:3] = d / n[:, None]
    u[:, 3] = l_c / n
    u[:, 4] = eps / n
    u[:, 5] = h_g / n
    u[:, 6:12] = np.asarray(S_c) / (M_c * l_c * l_c)[:, None]
    return u


def skip(u):
    """The fixed skip term 3 s of the outputs (s = the normalised second moments)."""
    return 3.0 * np.asarray(u, dtype=np.float64)[:, N_FEAT - N_OUT:N_FEAT]


def forward(p, u):
    """Returns (o [P,6], cache)."""
    z1 = u @ p["W1"] + p["b1"]
    h1 = gelu(z1)
    z2 = h1 @ p["W2"] + p["b2"]
    h2 = gelu(z2)
    o = h2 @ p["W3"] + p["b3"] + skip(u)
    return o, (u, z1, h1, z2, h2)


def gated_outputs(p, u, gate):
    """Outputs with the gate applied: the layers' part only where u[:, 3] >= gate."""
    o, _ = forward(p, u)
    off = np.asarray(u)[:, 3] < gate
    o[off] = skip(u[off])
    return o


def traceless(o):
    """P(o): subtract a third of the trace from the diagonal (xx, yy, zz)."""
    q = np.array(o, dtype=np.float64, copy=True)
    t = (q[:, 0] + q[:, 1] + q[:, 2]) / 3.0
    q[:, 0:3] -= t[:, None]
    return q


def quad_accel_basis(dvec, eps):
    """Linear map Qt -> a_Qt at offset d = x - COM.

    Returns B[P,3,6] with a_Qt = B @ (xx, yy, zz, xy, xz, yz), from
    a_Q = Q d r^-5 - 5/2 (d^T Q d) d r^-7, r^2 = |d|^2 + eps^2.
    """
    d = np.asarray(dvec, dtype=np.float64)
    r2 = (d * d).sum(axis=1) + eps * eps
    r5 = r2 ** -2.5
    r7 = r2 ** -3.5
    x, y, z = d[:, 0], d[:, 1], d[:, 2]
    # d^T Q d coefficients for (xx, yy, zz, xy, xz, yz)
    dqd = np.stack([x * x, y * y, z * z, 2 * x * y, 2 * x * z, 2 * y * z], axis=1)
    # Q d coefficients, row k of Q d
    qd = np.zeros((len(d), 3, 6))
    qd[:, 0, 0] = x
    qd[:, 0, 3] = y
    qd[:, 0, 4] = z
    qd[:, 1, 1] = y
    qd[:, 1, 3] = x
    qd[:, 1, 5] = z
    qd[:, 2, 2] = z
    qd[:, 2, 4] = x
    qd[:, 2, 5] = y
    return qd * r5[:, None, None] - 2.5 * d[:, :, None] * dqd[:, None, :] * r7[:, None, None]


def sample_weights(a_target, t, kept):
    """Training weights w = W / |a_i|^2 (a_target [P,3] the total force on
    each sample's target, t [P,3] the cell targets, kept [P] bool the gate's
    selection), W normalising the kept samples' mean of w |t|^2 to 1 (W = 1
    when every kept t is zero); |a_i|^2 is taken as at least 1e-300."""
    a2 = np.maximum((np.asarray(a_target, np.float64) ** 2).sum(axis=1), 1e-300)
    t2 = (np.asarray(t, np.float64) ** 2).sum(axis=1)
    kept = np.asarray(kept, bool)
    s = float(np.sum(t2[kept] / a2[kept]))
    W = kept.sum() / s if s > 0 else 1.0
    return W / a2


def loss(p, u, dvec, M_c, l_c, t, eps, w):
    """Mean weighted squared residual over samples (one network row each),
    weights w [P]."""
    o, _ = forward(p, u)
    q = traceless(o) * (M_c * l_c * l_c)[:, None]
    a_q = np.einsum("pkj,pj->pk", quad_accel_basis(dvec, eps), q)
    r = a_q - t
    return float(np.mean(np.asarray(w) * (r * r).sum(axis=1)))


def loss_and_grad(p, u, dvec, M_c, l_c, t, eps, w):
    """Loss and the gradient with respect to every parameter (hand reverse mode)."""
    P = len(u)
    o, (u_, z1, h1, z2, h2) = forward(p, u)
    scale = M_c * l_c * l_c
    B = quad_accel_basis(dvec, eps)
    q = traceless(o) * scale[:, None]
    a_q = np.einsum("pkj,pj->pk", B, q)
    r = a_q - t
    w = np.asarray(w, np.float64)
    L = float(np.mean(w * (r * r).sum(axis=1)))
    # dL/dr = 2 w r / P
    dr = (2.0 / P) * w[:, None] * r
    dq = np.einsum("pkj,pk->pj", B, dr) * scale[:, None]
    # through P: o_aa -> o_aa - tr/3 ; dL/do_aa = dq_aa - mean(dq_xx, dq_yy, dq_zz)
    do = dq.copy()
    m = (dq[:, 0] + dq[:, 1] + dq[:, 2]) / 3.0
    do[:, 0:3] -= m[:, None]
    g = {}
    g["W3"] = h2.T @ do
    g["b3"] = do.sum(axis=0)
    dh2 = do @ p["W3"].T
    dz2 = dh2 * gelu_grad(z2)
    g["W2"] = h1.T @ dz2
    g["b2"] = dz2.sum(axis=0)
    dh1 = dz2 @ p["W2"].T
    dz1 = dh1 * gelu_grad(z1)
    g["W1"] = u_.T @ dz1
    g["b1"] = dz1.sum(axis=0)
    return L, g, {"do": do, "dz2": dz2, "dz1": dz1}


def adam_step(p, g, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba 2015) with bias correction; returns new dicts."""
    out_p, out_m, out_v = {}, {}, {}
    for k in p:
        out_m[k] = beta1 * m[k] + (1 - beta1) * g[k]
        out_v[k] = beta2 * v[k] + (1 - beta2) * g[k] * g[k]
        mh = out_m[k] / (1 - beta1 ** step)
        vh = out_v[k] / (1 - beta2 ** step)
        out_p[k] = p[k] - lr * mh / (np.sqrt(vh) + eps)
    return out_p, out_m, out_v


def exact_quadrupole(S):
    """Textbook quadrupole tensor Q = 3 S - tr(S) I of a second-moment tensor."""
    S = np.asarray(S, dtype=np.float64)
    tr = S[:, 0] + S[:, 1] + S[:, 2]
    Q = 3.0 * S
    Q[:, 0:3] -= tr[:, None]
    return Q


def to_bf16(x):
    """Round to the nearest BF16 value (ties to even), returned as float64.

    BF16 keeps the top 16 bits of an FP32 word: round the FP32 value's low 16
    bits to nearest, ties to the even upper half.
    """
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    low = u & 0xFFFF
    up = u >> 16
    round_up = (low > 0x8000) | ((low == 0x8000) & ((up & 1) == 1))
    up = up + round_up.astype(np.uint64)
    return (up << 16).astype(np.uint32).view(np.float32).astype(np.float64)


def bf16_params(p):
    """Weights rounded to BF16, biases kept (the device keeps FP32 biases)."""
    q = dict(p)
    for k in ("W1", "W2", "W3"):
        q[k] = to_bf16(p[k])
    return q


def flat_to_params(v):
    """Parameter dict from the flat vector W1, b1, W2, b2, W3, b3 (row-major)."""
    v = np.asarray(v, dtype=np.float64)
    out, off = {}, 0
    for k, shape in (("W1", (N_IN, N_H)), ("b1", (N_H,)), ("W2", (N_H, N_H)), ("b2", (N_H,)),
                     ("W3", (N_H, N_OUT)), ("b3", (N_OUT,))):
        size = int(np.prod(shape))
        out[k] = v[off:off + size].reshape(shape)
        off += size
    assert off == len(v)
    return out


def params_to_flat(p):
    return np.concatenate([p[k].ravel() for k in ("W1", "b1", "W2", "b2", "W3", "b3")])


def expanded_basis(D, delta, eps):
    """Linear map Qt -> correction at x = c_g + delta through the second-order
    local expansion about c_g, where D = c_g - COM.

    B[P,3,6] such that a = B @ (xx, yy, zz, xy, xz, yz), with
    a = A + J delta + 1/2 H[delta, delta] and A, J, H the quadrupole-form field
    and its derivatives at c_g (oracle_quad_derivs).
    """
    import oracle
    D = np.asarray(D, dtype=np.float64).reshape(-1, 3)
    delta = np.asarray(delta, dtype=np.float64).reshape(-1, 3)
    P = len(D)
    hidx = [(0, 0, 0), (1, 1, 1), (2, 2, 2), (0, 0, 1), (0, 0, 2), (0, 1, 1), (1, 1, 2), (0, 2, 2), (1, 2, 2),
            (0, 1, 2)]
    B = np.zeros((P, 3, 6))
    for m in range(6):
        e = np.zeros((P, 6))
        e[:, m] = 1.0
        A, J6, H10, _ = oracle.quad_derivs(D, np.zeros((P, 3)), e, eps)
        J = np.zeros((P, 3, 3))
        for k, (i, j) in enumerate(((0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2))):
            J[:, i, j] = J6[:, k]
            J[:, j, i] = J6[:, k]
        H = np.zeros((P, 3, 3, 3))
        import itertools
        for k, (i, j, l) in enumerate(hidx):
            for perm in set(itertools.permutations((i, j, l))):
                H[:, perm[0], perm[1], perm[2]] = H10[:, k]
        B[:, :, m] = (A + np.einsum("pij,pj->pi", J, delta)
                      + 0.5 * np.einsum("pijk,pj,pk->pi", H, delta, delta))
    return B


def loss_and_grad_basis(p, u, B, scale, t, w, return_cache=False):
    """Mean of w |B (scale P(o)) - t|^2 over samples and its parameter gradient.

    Same reverse mode as ``loss_and_grad`` with the applied map B given.  With
    ``return_cache`` also the forward activations and backward signals
    {h1, h2, do, dz2, dz1}.
    """
    P = len(u)
    o, (u_, z1, h1, z2, h2) = forward(p, u)
    q = traceless(o) * scale[:, None]
    r = np.einsum("pkj,pj->pk", B, q) - t
    L = float(np.mean(w * (r * r).sum(axis=1)))
    dr = (2.0 / P) * w[:, None] * r
    dq = np.einsum("pkj,pk->pj", B, dr) * scale[:, None]
    do = dq.copy()
    m = (dq[:, 0] + dq[:, 1] + dq[:, 2]) / 3.0
    do[:, 0:3] -= m[:, None]
    g = {}
    g["W3"] = h2.T @ do
    g["b3"] = do.sum(axis=0)
    dh2 = do @ p["W3"].T
    dz2 = dh2 * gelu_grad(z2)
    g["W2"] = h1.T @ dz2
    g["b2"] = dz2.sum(axis=0)
    dh1 = dz2 @ p["W2"].T
    dz1 = dh1 * gelu_grad(z1)
    g["W1"] = u_.T @ dz1
    g["b1"] = dz1.sum(axis=0)
    if return_cache:
        return L, g, {"u": u_, "h1": h1, "h2": h2, "do": do, "dz2": dz2, "dz1": dz1}
    return L, g
