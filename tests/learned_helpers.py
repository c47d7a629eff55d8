"""Test helpers for the cell-correction parity tests (index bookkeeping and
the truncation bound of the local expansion); no arithmetic of the method.

Truncation bound.  For a traceless symmetric tensor Q the quadrupole-form
potential about a cell's centre of mass is
    phi(x) = -1/2 d.Q d r^-5 = -(1/6) Q : grad grad (1/r),
    d = x - COM,  r^2 = |d|^2 + eps^2,
since grad grad (1/r) = (3 d d^T - r^2 I) r^-5 and Q has no trace.  With
(d, eps) read as a point of R^4 and u a unit vector of R^3, 1/r is
1 / |(d, eps)|, and the generating function of the Legendre polynomials
gives the m-th derivative along u as m! P_m(cos) / r^(m+1), so its size is
at most m! / r^(m+1); by Banach's theorem on symmetric multilinear forms
over a Hilbert space the same bound holds for every mixed derivative along
unit vectors u_1 .. u_m.  Writing Q = sum_k lambda_k e_k e_k^T:
    |grad^3 a [v, u, u, u]| <= (1/6) sum_k |lambda_k| 6! / r^7
                             = 120 ||Q||_* / r^7,
    |grad^3 phi [u, u, u]|  <= (1/6) ||Q||_* 5! / r^6 = 20 ||Q||_* / r^6,
with ||Q||_* the sum of |eigenvalues|.  The second-order Taylor expansion
about the group's box centre c_g, evaluated at x = c_g + delta, leaves the
integral remainder of size at most (1/6) |delta|^3 times the third-derivative
bound taken on the segment from c_g to x, whose points are at least the
point-segment distance d_seg from the COM:
    |R_a|   <= 20 ||Q||_* |delta|^3 / rho^7,
    |R_phi| <= (10/3) ||Q||_* |delta|^3 / rho^6,
    rho^2 = d_seg^2 + eps^2.
Summed over a group's cells this bounds, per target, the difference between
the per-particle quadrupole form and its local expansion.
"""
import numpy as np


def group_geometry(pos, group_off):
    """Bounding-box centre [G,3] and half-diagonal [G] of each group (FP64)."""
    pos = np.asarray(pos, np.float64)
    go = np.asarray(group_off, np.int64)
    lo = np.minimum.reduceat(pos, go[:-1], axis=0)
    hi = np.maximum.reduceat(pos, go[:-1], axis=0)
    return 0.5 * (lo + hi), 0.5 * np.linalg.norm(hi - lo, axis=1)


def pair_counts(lists):
    """(group, cell) pairs per group: the near cells of a walk that listed
    them first, else every cell entry."""
    return np.asarray(getattr(lists, "n_pair", lists.n_cellent), np.int64)


def pair_index(lists, n):
    """Group and cell (0-based cell number) of every (group, cell) pair, in pair order."""
    nce = pair_counts(lists)
    G = len(nce)
    g = np.repeat(np.arange(G), nce)
    pair_off = np.concatenate([[0], np.cumsum(nce)])
    within = np.arange(pair_off[-1]) - np.repeat(pair_off[:-1], nce)
    c = np.asarray(lists.list_idx, np.int64)[np.asarray(lists.list_off, np.int64)[g] + within] - n
    return g, c


def group_of(group_off, i):
    return np.searchsorted(np.asarray(group_off, np.int64), np.asarray(i, np.int64), side="right") - 1


def pair_cells(lists, n, pairs):
    """Group and cell (0-based) of the given global pair numbers."""
    pair_off = np.concatenate([[0], np.cumsum(pair_counts(lists))])
    pairs = np.asarray(pairs, np.int64)
    g = np.searchsorted(pair_off, pairs, side="right") - 1
    c = np.asarray(lists.list_idx, np.int64)[np.asarray(lists.list_off, np.int64)[g] + pairs - pair_off[g]] - n
    return g, c


def sample_groups(lists, n_groups, per_group, seed):
    """`n_groups` distinct groups (ascending) and up to `per_group` targets of
    each (evenly spaced in the group), drawn with a seeded generator."""
    rng = np.random.default_rng(seed)
    groups = np.sort(rng.choice(lists.n_groups, min(n_groups, lists.n_groups), replace=False))
    go = np.asarray(lists.group_off, np.int64)
    tgt = []
    for g in groups:
        ids = np.arange(go[g], go[g + 1])
        step = max(1, len(ids) // per_group)
        tgt.append(ids[::step][:per_group])
    return groups, np.concatenate(tgt).astype(np.int64)


def sub_lists(lists, groups):
    """The CSR restricted to `groups` (ascending), other particle ranges kept
    as groups with empty lists, so that every particle still has a group.
    Returns dict(group_off, list_off, list_idx, n_cellent, pairs) with
    n_cellent the kept groups' pair counts (the cells that carry a tensor)
    and `pairs` the global pair numbers of their pairs, in the restricted
    pair order."""
    go = np.asarray(lists.group_off, np.int64)
    lo = np.asarray(lists.list_off, np.int64)
    li = np.asarray(lists.list_idx, np.int64)
    nce = pair_counts(lists)
    pair_off = np.concatenate([[0], np.cumsum(nce)])
    groups = np.unique(np.asarray(groups, np.int64))
    bounds, lens, ncs, idx, pairs = [int(go[0])], [], [], [], []
    for g in groups:
        if go[g] > bounds[-1]:          # the particles before this group: a group with an empty list
            bounds.append(int(go[g]))
            lens.append(0)
            ncs.append(0)
        bounds.append(int(go[g + 1]))
        lens.append(int(lo[g + 1] - lo[g]))
        ncs.append(int(nce[g]))
        idx.append(li[lo[g]:lo[g + 1]])
        pairs.append(np.arange(pair_off[g], pair_off[g + 1]))
    if go[-1] > bounds[-1]:
        bounds.append(int(go[-1]))
        lens.append(0)
        ncs.append(0)
    return dict(group_off=np.array(bounds, np.int64), list_off=np.concatenate([[0], np.cumsum(lens)]).astype(np.int64),
                list_idx=np.concatenate(idx).astype(np.int64), n_cellent=np.array(ncs, np.int64),
                pairs=np.concatenate(pairs).astype(np.int64))


def sym6_to_mat(q6):
    q6 = np.asarray(q6, np.float64)
    m = np.empty(q6.shape[:-1] + (3, 3))
    m[..., 0, 0], m[..., 1, 1], m[..., 2, 2] = q6[..., 0], q6[..., 1], q6[..., 2]
    m[..., 0, 1] = m[..., 1, 0] = q6[..., 3]
    m[..., 0, 2] = m[..., 2, 0] = q6[..., 4]
    m[..., 1, 2] = m[..., 2, 1] = q6[..., 5]
    return m


def nuclear_norm6(q6):
    """Sum of |eigenvalues| of symmetric tensors given as (xx, yy, zz, xy, xz, yz)."""
    return np.abs(np.linalg.eigvalsh(sym6_to_mat(q6))).sum(axis=-1)


def segment_distance(p, a, b):
    """Distance from points p [..., 3] to the segments [a, b] (broadcast)."""
    ab = np.asarray(b) - np.asarray(a)
    ap = np.asarray(p) - np.asarray(a)
    den = (ab * ab).sum(axis=-1)
    t = np.clip(np.where(den > 0, (ap * ab).sum(axis=-1) / np.where(den > 0, den, 1.0), 0.0), 0.0, 1.0)
    return np.linalg.norm(ap - t[..., None] * ab, axis=-1)


def truncation_bound(x, centre, com, qnorm, eps):
    """Bounds (acc, pot) on the truncation error at points x [T,3] of the
    second-order expansion about centre [T,3] of the quadrupole-form fields
    of tensors with nuclear norms qnorm [T,C] at com [T,C,3] (zero norms pad
    short lists)."""
    x = np.asarray(x, np.float64)
    centre = np.asarray(centre, np.float64)
    delta = np.linalg.norm(x - centre, axis=1)[:, None]
    ds = segment_distance(np.asarray(com), centre[:, None, :], x[:, None, :])
    rho2 = ds ** 2 + eps * eps
    ba = (20.0 * qnorm * delta ** 3 / rho2 ** 3.5).sum(axis=1)
    bp = (10.0 / 3.0 * qnorm * delta ** 3 / rho2 ** 3).sum(axis=1)
    return ba, bp


def target_bounds(pos, group_off, centre, tgt, lists_sub, com_of_cell, qnorm_of_pair, n, eps, qtol_of_pair=None):
    """Per-target truncation bounds for targets `tgt` (particle indices) over
    their groups' cells in a restricted CSR from `sub_lists` (qnorm_of_pair
    indexed like lists_sub['pairs']).  With qtol_of_pair (bounds on the
    nuclear norm of each tensor's error) also the bounds on the field and
    potential of those errors at the target, sum ||dQ||_* / r^4 and
    sum ||dQ||_* / (3 r^3) (|a_Q| <= ||Q||_* / r^4 and |phi_Q| <= ||Q||_* / (3 r^3)
    by the derivative bound above with m = 3 and 2), as two more arrays."""
    go = lists_sub["group_off"]
    lo, li, nce = lists_sub["list_off"], lists_sub["list_idx"], lists_sub["n_cellent"]
    sub_pair_off = np.concatenate([[0], np.cumsum(nce)])
    gfull = group_of(group_off, tgt)
    gsub = group_of(go, tgt)
    ba = np.empty(len(tgt))
    bp = np.empty(len(tgt))
    bt = np.zeros(len(tgt))
    btp = np.zeros(len(tgt))
    for k, (i, g, s) in enumerate(zip(tgt, gfull, gsub)):
        cells = li[lo[s]:lo[s] + nce[s]] - n
        qn = qnorm_of_pair[sub_pair_off[s]:sub_pair_off[s + 1]]
        a, p = truncation_bound(pos[i][None], centre[g][None], com_of_cell[cells][None], qn[None], eps)
        ba[k], bp[k] = a[0], p[0]
        if qtol_of_pair is not None:
            r2 = ((pos[i] - com_of_cell[cells]) ** 2).sum(axis=1) + eps * eps
            qt = qtol_of_pair[sub_pair_off[s]:sub_pair_off[s + 1]]
            bt[k] = np.sum(qt / r2 ** 2)
            btp[k] = np.sum(qt / (3.0 * r2 ** 1.5))
    if qtol_of_pair is not None:
        return ba, bp, bt, btp
    return ba, bp
