"""Oracle side of the cell-correction parity tests: per-pair tensors of the
FP64 oracle (textbook quadrupole or the network at BF16-rounded weights and
features), their BF16 error allowance, and the comparison of a device force
with the oracle's list force in both applied forms (second-order local
expansion, and the per-particle quadrupole form that defines the
correction)."""
import numpy as np

import oracle
from oracle import mlp as omlp
from learned_helpers import group_geometry, nuclear_norm6, pair_cells, sub_lists, sym6_to_mat, target_bounds

# Relative size of the BF16 rounding of the network (weights, features and
# hidden activations rounded to BF16, unit roundoff 2^-8; a few roundings
# compound through three layers) against the absolute-value scale of each
# quantity: 5 unit roundoffs.
BF16_TOL = 2e-2


def abs_scale_outputs(p, u, cache):
    """Per-row, per-output scale sum_j |h2_j W3_jk| + |b3_k| + |skip_k| of the
    network outputs: the size the BF16 errors are relative to."""
    h2 = cache[4]
    return np.abs(h2) @ np.abs(p["W3"]) + np.abs(p["b3"]) + np.abs(omlp.skip(u))


def projected_scale(so):
    """Entry-wise scale of P(o) from the scale of o (P removes a third of the trace)."""
    out = np.array(so, dtype=np.float64, copy=True)
    out[:, 0:3] += (so[:, 0] + so[:, 1] + so[:, 2])[:, None] / 3.0
    return out


def pair_tensors(kind, lists, pos32, cm, eps, pairs, params=None, gate=0.0):
    """(Q [P,6], tolerance [P,6]) of the oracle for the given global pairs:
    kind "quad" the textbook tensor 3 S - tr(S) I (no tolerance), kind "mlp"
    the network's tensor M l^2 P(o) at BF16 weights and features with the
    gate applied, and BF16_TOL times the entry-wise scale of the gated
    pairs' tensors."""
    n = len(pos32)
    g, c = pair_cells(lists, n, pairs)
    cmd = cm.astype(np.float64)
    if kind == "quad":
        Q = omlp.exact_quadrupole(cmd[c, 5:11])
        return Q, np.zeros_like(Q)
    centre, hdiag = group_geometry(pos32.astype(np.float64), lists.group_off)
    M, l = cmd[c, 3], cmd[c, 4]
    u = omlp.to_bf16(omlp.features(cmd[c, :3] - centre[g], l, float(np.float32(eps)), hdiag[g], cmd[c, 5:11], M))
    p = omlp.bf16_params(omlp.flat_to_params(params))
    o, cache = omlp.forward(p, u)
    on = u[:, 3] >= gate
    o[~on] = omlp.skip(u[~on])
    scale = M * l * l
    Q = omlp.traceless(o) * scale[:, None]
    tol = BF16_TOL * projected_scale(abs_scale_outputs(p, u, cache)) * scale[:, None]
    tol[~on] = 0.0
    return Q, tol


def frob_sym6(t6):
    t6 = np.asarray(t6, np.float64)
    return np.sqrt((t6[:, :3] ** 2).sum(axis=1) + 2.0 * (t6[:, 3:] ** 2).sum(axis=1))


def compare(dev_acc, dev_pot, pos32, mass32, lists, cm, eps, tgt, groups, kind, params=None, gate=0.0,
            med_bar=1e-6, p99_bar=1e-5, max_bar=1e-4, label=""):
    """Device accelerations/potentials at targets `tgt` (rows of the full
    device outputs) against the oracle's list force with the same tensors:
      1. element by element against the expanded form (the FP32 parity: the
         device computes exactly this), median <= med_bar, 99th percentile
         <= p99_bar;
      2. per target against the per-particle quadrupole form (the definition):
         |a_dev - a_def| <= B_i + T_i + max_bar |a_def|, with B_i the
         truncation bound of the expansion and T_i the field of the tensors'
         BF16 allowance, and the median relative deviation at most 1.5 times
         the truncation the oracle itself measures (expanded against
         per-particle) plus med_bar.
    Returns a dict of the statistics."""
    n = len(mass32)
    sub = sub_lists(lists, groups)
    Q, Qtol = pair_tensors(kind, lists, pos32, cm, eps, sub["pairs"], params, gate)
    p64, m64 = pos32.astype(np.float64), mass32.astype(np.float64)
    cmd = cm.astype(np.float64)
    e = float(np.float32(eps))
    args = (p64, m64, sub["group_off"], sub["list_off"], sub["list_idx"], cmd[:, :3], cmd[:, 3], e)
    a_def, p_def = oracle.list_force(*args, tgt=tgt, n_cellent=sub["n_cellent"], quad=Q)
    a_exp, p_exp = oracle.list_force(*args, tgt=tgt, n_cellent=sub["n_cellent"], quad=Q, expanded=True)
    a_dev = np.asarray(dev_acc, np.float64)[tgt]
    p_dev = np.asarray(dev_pot, np.float64)[tgt]
    ea = oracle.rel_err(a_dev, a_exp)
    ep = oracle.rel_err(p_dev, p_exp)
    centre, _ = group_geometry(p64, lists.group_off)
    ba, bp, bt, btp = target_bounds(p64, lists.group_off, centre, tgt, sub, cmd[:, :3], nuclear_norm6(Q), n, e,
                               qtol_of_pair=np.sqrt(3.0) * frob_sym6(Qtol))
    an = np.linalg.norm(a_def, axis=1)
    d = np.linalg.norm(a_dev - a_def, axis=1)
    trunc = np.linalg.norm(a_exp - a_def, axis=1) / an
    dev_rel = d / an
    st = dict(exp_acc_median=float(np.median(ea)), exp_acc_p99=float(np.quantile(ea, 0.99)),
              exp_pot_median=float(np.median(ep)), def_acc_median=float(np.median(dev_rel)),
              def_acc_max=float(dev_rel.max()), trunc_median=float(np.median(trunc)),
              bound_median=float(np.median(ba / an)), slack_min=float(np.min((ba + bt + max_bar * an - d) / an)))
    print(f"{label}: vs expanded oracle acc median {st['exp_acc_median']:.2e} p99 {st['exp_acc_p99']:.2e} pot "
          f"median {st['exp_pot_median']:.2e} | vs per-particle form median {st['def_acc_median']:.2e} max "
          f"{st['def_acc_max']:.2e} (oracle truncation median {st['trunc_median']:.2e}, bound median "
          f"{st['bound_median']:.2e})", flush=True)
    assert st["exp_acc_median"] <= med_bar and st["exp_acc_p99"] <= p99_bar and st["exp_pot_median"] <= med_bar, st
    assert np.all(d <= ba + bt + max_bar * an), st
    assert np.all(np.abs(p_dev - p_def) <= bp + btp + max_bar * np.abs(p_def)), st
    assert st["def_acc_median"] <= 1.5 * st["trunc_median"] + med_bar, st
    return st
