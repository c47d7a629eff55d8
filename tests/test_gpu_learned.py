"""GPU parity of the learned cell correction against the FP64 network oracle.

The device runs the network with BF16 operands (weights, features and hidden
activations rounded to BF16) and FP32 accumulation; the oracle runs in FP64 at
the same BF16-rounded weights and inputs, so the remaining difference is the
rounding of hidden activations and of the FP32 sums: relative L2 <= 2e-2 per
tensor.  Training targets are FP64 sums on both sides (1e-5 of |t|).
"""
import numpy as np
import pytest

import oracle
import synth
import paper_1206_1199_amd as otoo
from oracle import mlp as omlp

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
learned = pytest.importorskip("paper_1206_1199_amd.learned")

EPS = 0.01


def rel_l2(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def bf16_bits_to_f64(X):
    b = X.cpu().numpy().view(np.uint16).astype(np.uint32) << 16
    return b.view(np.float32).astype(np.float64)


@pytest.fixture(scope="module")
def env():
    ctx = otoo.Context(0)
    net = learned.Network(ctx)
    pos, m = synth.plummer(16384, seed=0)
    tree = otoo.Tree(pos, m, n_crit=16)
    lists = tree.walk(theta=0.7, g_max=64)
    d, first, count = learned.device_tree_arrays(tree, lists)
    _, pos32, mass32, cm = tree.export(12)
    cells = tree.cells()
    rng = np.random.default_rng(40)
    samples = learned.draw_samples(lists, 3000, rng)
    params = learned.init_params(7)
    net.set_params(params)
    X, aux = net.train_samples(d, first, count, EPS, torch.from_numpy(samples).cuda())
    torch.cuda.synchronize()
    ctx.check()
    return dict(ctx=ctx, net=net, tree=tree, lists=lists, d=d, pos32=pos32, mass32=mass32, cm=cm, cells=cells,
                samples=samples, params=params, X=X, aux=aux)


def _pair_cell(lists, n, p):
    g = np.searchsorted(lists.pair_off, p, side="right") - 1
    k = p - lists.pair_off[g]
    return g, lists.list_idx[lists.list_off[g] + k] - n


def _group_geometry(pos32, lists, g):
    pts = pos32[lists.group_off[g]:lists.group_off[g + 1]].astype(np.float64)
    lo, hi = pts.min(0), pts.max(0)
    return 0.5 * (lo + hi), 0.5 * np.linalg.norm(hi - lo)


def test_train_samples_match_exact_cell_sums(env):
    lists, cm, pos32, mass32 = env["lists"], env["cm"], env["pos32"], env["mass32"]
    n = len(mass32)
    aux = env["aux"].cpu().numpy().astype(np.float64)
    X = bf16_bits_to_f64(env["X"])
    first, count = env["cells"]["first"], env["cells"]["count"]
    sel = np.arange(0, len(env["samples"]), 7)
    t_ref, D_ref, del_ref, feat_ref, mono_ref = [], [], [], [], []
    for s in sel:
        p, i = env["samples"][s]
        g, c = _pair_cell(lists, n, p)
        cg, h = _group_geometry(pos32, lists, g)
        ids = np.arange(first[c], first[c] + count[c])
        x = pos32[i].astype(np.float64)
        a_ex, _ = oracle.point_field(x[None], [0, len(ids)], ids, pos32.astype(np.float64),
                                     mass32.astype(np.float64), float(np.float32(EPS)))
        com = cm[c, :3].astype(np.float64)
        a_mo, _ = oracle.point_field(x[None], [0, 1], [0], com[None], cm[c, 3:4].astype(np.float64),
                                     float(np.float32(EPS)))
        t_ref.append(a_ex[0] - a_mo[0])
        mono_ref.append(np.linalg.norm(a_mo[0]))
        D_ref.append(cg - com)
        del_ref.append(x - cg)
        feat_ref.append(omlp.features((com - cg)[None], cm[c, 4:5].astype(np.float64), float(np.float32(EPS)),
                                      np.array([h]), cm[c, 5:11][None].astype(np.float64),
                                      cm[c, 3:4].astype(np.float64))[0])
    t_ref, D_ref, del_ref, feat_ref, mono_ref = map(np.array, (t_ref, D_ref, del_ref, feat_ref, mono_ref))
    # t is a small difference of FP64 sums stored in FP32: within FP32 rounding
    # of t plus FP64 rounding of the monopole-sized sums (a one-particle cell
    # has t = 0 up to that rounding)
    dt = np.linalg.norm(aux[sel, 6:9] - t_ref, axis=1)
    tn = np.linalg.norm(t_ref, axis=1)
    assert np.all(dt <= 1e-7 * tn + 1e-12 * mono_ref)
    nz = tn > 1e-9 * mono_ref
    err_t = dt[nz] / tn[nz]
    print(f"targets: median rel err {np.median(err_t):.2e}, max {err_t.max():.2e}, one-particle {np.sum(~nz)}",
          flush=True)
    assert np.median(err_t) <= 1e-6
    scale = np.abs(D_ref).max()
    np.testing.assert_allclose(aux[sel, 0:3], D_ref, atol=1e-6 * scale)
    np.testing.assert_allclose(aux[sel, 3:6], del_ref, atol=1e-6 * scale)
    # features: the device rounds its FP32 features to BF16
    np.testing.assert_allclose(X[sel, :12], feat_ref[:, :12], rtol=2 ** -7, atol=1e-6)
    assert np.all(X[:, 12:] == 0)


def test_forward_matches_oracle(env):
    out = env["net"].forward(env["X"]).cpu().numpy()
    p = omlp.bf16_params(omlp.flat_to_params(env["params"]))
    o_ref, _ = omlp.forward(p, bf16_bits_to_f64(env["X"]))
    e = rel_l2(out, o_ref)
    print(f"forward rel L2 {e:.2e}", flush=True)
    assert e <= 2e-2


def _oracle_loss_grad(env, params):
    aux = env["aux"].cpu().numpy().astype(np.float64)
    B = omlp.expanded_basis(aux[:, 0:3], aux[:, 3:6], float(np.float32(EPS)))
    p = omlp.bf16_params(omlp.flat_to_params(params))
    return omlp.loss_and_grad_basis(p, bf16_bits_to_f64(env["X"]), B, aux[:, 9], aux[:, 6:9], aux[:, 10])


def test_backward_matches_oracle(env):
    net = env["net"]
    rng = np.random.default_rng(3)
    params = env["params"] + rng.normal(size=env["params"].shape).astype(np.float32) * 0.05
    net.set_params(params)
    g, L = net.backward(env["X"], env["aux"], EPS)
    L_ref, g_ref = _oracle_loss_grad(env, params)
    gd = omlp.flat_to_params(g)
    print(f"loss {L:.6e} oracle {L_ref:.6e}", flush=True)
    assert L == pytest.approx(L_ref, rel=1e-2)
    for k in g_ref:
        e = rel_l2(gd[k], g_ref[k])
        print(f"grad {k}: rel L2 {e:.2e}", flush=True)
        assert e <= 2e-2, k
    net.set_params(env["params"])


def test_adam_step_matches_oracle(env):
    net = env["net"]
    net.set_params(env["params"])
    g, _ = net.backward(env["X"], env["aux"], EPS)
    net.train_step(env["X"], env["aux"], EPS, 1e-3)
    p1, m1, v1, step = net.get_params()
    assert step == 1
    p0 = omlp.flat_to_params(env["params"].astype(np.float64))
    gd = omlp.flat_to_params(g.astype(np.float64))
    z = {k: np.zeros_like(v) for k, v in p0.items()}
    pr, mr, vr = omlp.adam_step(p0, gd, z, z, 1, 1e-3)
    np.testing.assert_allclose(p1, omlp.params_to_flat(pr), rtol=1e-6, atol=1e-7)
    np.testing.assert_allclose(m1, omlp.params_to_flat(mr), rtol=1e-6, atol=1e-12)
    np.testing.assert_allclose(v1, omlp.params_to_flat(vr), rtol=1e-5, atol=1e-18)
    net.set_params(env["params"])


def test_checkpoint_resume_is_exact(env, tmp_path):
    net, X, aux = env["net"], env["X"], env["aux"]
    net.set_params(env["params"])
    for _ in range(3):
        net.train_step(X, aux, EPS, 1e-3)
    path = tmp_path / "net.ckpt"
    net.save(path)
    for _ in range(3):
        net.train_step(X, aux, EPS, 1e-3)
    pa = net.get_params()
    net2 = learned.Network(env["ctx"])
    net2.load(path)
    for _ in range(3):
        net2.train_step(X, aux, EPS, 1e-3)
    pb = net2.get_params()
    for a, b in zip(pa[:3], pb[:3]):
        np.testing.assert_array_equal(a, b)
    assert pa[3] == pb[3] == 6
    net.set_params(env["params"])


@pytest.mark.parametrize("gate", [0.0, 0.4])
def test_infer_matches_oracle(env, gate):
    """Per-pair tensors (skip term plus the layers where the gate lets them
    run) against the oracle network at the same BF16 features."""
    net, d, lists, cm, pos32 = env["net"], env["d"], env["lists"], env["cm"], env["pos32"]
    net.set_params(env["params"])
    net.set_gate(gate)
    try:
        corr = net.infer(d, EPS).cpu().numpy().astype(np.float64)
    finally:
        net.set_gate(0.0)
    env["ctx"].check()
    n = len(pos32)
    sel = np.arange(0, int(lists.pair_off[-1]), 11)
    feats, scale = [], []
    for p in sel:
        g, c = _pair_cell(lists, n, p)
        cg, h = _group_geometry(pos32, lists, g)
        com = cm[c, :3].astype(np.float64)
        feats.append(omlp.features((com - cg)[None], cm[c, 4:5].astype(np.float64), float(np.float32(EPS)),
                                   np.array([h]), cm[c, 5:11][None].astype(np.float64),
                                   cm[c, 3:4].astype(np.float64))[0])
        scale.append(float(cm[c, 3]) * float(cm[c, 4]) ** 2)
    u = omlp.to_bf16(np.array(feats))
    o = omlp.gated_outputs(omlp.bf16_params(omlp.flat_to_params(env["params"])), u, gate)
    q_ref = omlp.traceless(o) * np.array(scale)[:, None]
    e = rel_l2(corr[sel], q_ref)
    frac = np.mean(u[:, 3] >= gate)
    print(f"inference gate {gate} ({frac:.2f} of pairs through the layers): rel L2 {e:.2e}", flush=True)
    assert e <= 3e-2
    if gate > 0:
        assert 0.05 < frac < 0.95
        off = u[:, 3] < gate          # the skip term alone: the textbook quadrupole of the BF16 moments
        np.testing.assert_allclose(corr[sel][off], q_ref[off], rtol=1e-5, atol=1e-6 * np.abs(q_ref).max())


def test_training_reduces_loss_and_helps_forces(env):
    ctx, net = env["ctx"], env["net"]
    cfgs = [learned.SampleConfig("plummer", 16384, 1000 + k, EPS, th, 64, 60000)
            for k, th in enumerate((0.5, 0.6, 0.7, 0.8, 0.9, 0.75))]
    gate = 0.4
    X, aux, eps_all = learned.make_training_set(ctx, net, cfgs, seed=1, gate=gate)
    Xv, auxv, epsv = learned.make_training_set(
        ctx, net, [learned.SampleConfig("plummer", 16384, 1100, EPS, 0.8, 64, 30000)], seed=2, gate=gate)
    base = learned.zero_correction_loss(auxv)
    net.set_params(np.zeros(learned.N_PARAMS, np.float32))     # zero layers: the textbook quadrupole
    quad = learned.evaluate_loss(net, Xv, auxv, epsv)
    net.set_params(learned.init_params(0))
    learned.fit(net, X, aux, eps_all, steps=600, batch=16384, lr=2e-3, seed=0)
    val = learned.evaluate_loss(net, Xv, auxv, epsv)
    print(f"validation loss {val:.4e} vs plain monopole {base:.4e}, textbook quadrupole {quad:.4e}", flush=True)
    assert val < 0.5 * base
    assert val < quad
    # forces on a held-out Plummer sphere at theta = 0.8
    pos, m = synth.plummer(16384, seed=1101)
    tree = otoo.Tree(pos, m, n_crit=16)
    lists = tree.walk(theta=0.8, g_max=64)
    d, _, _ = learned.device_tree_arrays(tree, lists)
    _, pos32, mass32, _ = tree.export(12)
    net.set_gate(gate)
    gc = ctx.correction(d, otoo.CORR_MLP, EPS, net=net)
    net.set_gate(0.0)
    a_l, _ = ctx.force(d, EPS, gcorr=gc)
    a_q, _ = ctx.force(d, EPS, gcorr=ctx.correction(d, otoo.CORR_QUAD, EPS))
    a_m, _ = ctx.force(d, EPS)
    torch.cuda.synchronize()
    ctx.check()
    sample = synth.sample_idx(16384, 1024, seed=103)
    a_dir, _ = oracle.direct(pos32.astype(np.float64), mass32.astype(np.float64), float(np.float32(EPS)),
                             tgt=sample)
    e_l = np.median(oracle.rel_err(a_l.cpu().numpy()[sample], a_dir))
    e_m = np.median(oracle.rel_err(a_m.cpu().numpy()[sample], a_dir))
    e_q = np.median(oracle.rel_err(a_q.cpu().numpy()[sample], a_dir))
    print(f"theta 0.8 held out: monopole median {e_m:.2e}, quadrupole {e_q:.2e}, learned {e_l:.2e}", flush=True)
    assert e_l < 0.8 * e_m
    assert e_l < 1.05 * e_q


@pytest.mark.parametrize("net_kernel,gate", [(0, 0.0), (1, 0.0), (0, 0.4), (1, 0.4)])
def test_fused_learned_correction_matches_oracle(env, net_kernel, gate):
    """The fused per-group learned correction (register-resident network, or
    the LDS-staged one) against the oracle's list force with the oracle
    network's tensors (FP64 features rounded to BF16, BF16 weights): the
    tensors differ by the BF16 activations (~3e-3 relative), and the
    correction is a small part of the force."""
    ctx, net, d, lists, cm, pos32, mass32 = (env[k] for k in ("ctx", "net", "d", "lists", "cm", "pos32", "mass32"))
    net.set_params(env["params"])
    old = ctx.tuning()
    ctx.set_tuning(net_kernel=net_kernel)
    net.set_gate(gate)
    try:
        gc = ctx.correction(d, otoo.CORR_MLP, EPS, net=net)
    finally:
        ctx.set_tuning(chunk=old.chunk, blocks_per_cu=old.blocks_per_cu, lpt=old.lpt, tile=old.tile,
                       net_kernel=old.net_kernel)
        net.set_gate(0.0)
    acc, pot = ctx.force(d, EPS, gcorr=gc)
    torch.cuda.synchronize()
    ctx.check()
    n = len(pos32)
    feats, scale = [], []
    for p in range(int(lists.pair_off[-1])):
        g, c = _pair_cell(lists, n, p)
        cg, h = _group_geometry(pos32, lists, g)
        com = cm[c, :3].astype(np.float64)
        feats.append(omlp.features((com - cg)[None], cm[c, 4:5].astype(np.float64), float(np.float32(EPS)),
                                   np.array([h]), cm[c, 5:11][None].astype(np.float64),
                                   cm[c, 3:4].astype(np.float64))[0])
        scale.append(float(cm[c, 3]) * float(cm[c, 4]) ** 2)
    o = omlp.gated_outputs(omlp.bf16_params(omlp.flat_to_params(env["params"])), omlp.to_bf16(np.array(feats)),
                           gate)
    quad = omlp.traceless(o) * np.array(scale)[:, None]
    sample = synth.sample_idx(n, 2048, seed=7)
    a_ref, p_ref = oracle.list_force(pos32.astype(np.float64), mass32.astype(np.float64), lists.group_off,
                                     lists.list_off, lists.list_idx, cm[:, :3].astype(np.float64),
                                     cm[:, 3].astype(np.float64), float(np.float32(EPS)), tgt=sample,
                                     n_cellent=lists.n_cellent, quad=quad, expanded=True)
    ea = oracle.rel_err(acc.cpu().numpy().astype(np.float64)[sample], a_ref)
    ep = oracle.rel_err(pot.cpu().numpy()[sample], p_ref)
    print(f"fused learned correction (kernel {net_kernel}, gate {gate}): acc median {np.median(ea):.2e} "
          f"p99 {np.quantile(ea, 0.99):.2e}, "
          f"pot median {np.median(ep):.2e}", flush=True)
    assert np.median(ea) <= 2e-5 and np.quantile(ea, 0.99) <= 2e-4
    assert np.median(ep) <= 2e-5


@pytest.mark.parametrize("gate", [0.0, 0.3])
def test_queue_rounds_on_long_lists(env, gate):
    """Groups of 256 at theta 0.5 hold thousands of cells, so the register-
    resident kernel's queue of gated pairs runs many rounds and carries a
    remainder between them.  Its per-group expansion must match the
    LDS-staged kernel's, which runs every pair through the layers in order
    (the gate applied afterwards) with no queue."""
    ctx, net = env["ctx"], env["net"]
    net.set_params(env["params"])
    pos, m = synth.plummer(1 << 17, seed=41)
    tree = otoo.Tree(pos, m, n_crit=16)
    lists = tree.walk(theta=0.5, g_max=256)
    d, _, _ = learned.device_tree_arrays(tree, lists)
    cells_per_group = np.diff(lists.pair_off)
    print(f"cells per group: median {np.median(cells_per_group):.0f}, max {cells_per_group.max()}", flush=True)
    assert np.median(cells_per_group) > 2048
    old = ctx.tuning()
    out = {}
    net.set_gate(gate)
    try:
        for k in (0, 1):
            ctx.set_tuning(net_kernel=k)
            out[k] = ctx.correction(d, otoo.CORR_MLP, EPS, net=net).cpu().numpy().astype(np.float64)
    finally:
        net.set_gate(0.0)
        ctx.set_tuning(chunk=old.chunk, blocks_per_cu=old.blocks_per_cu, lpt=old.lpt, tile=old.tile,
                       net_kernel=old.net_kernel)
    ctx.check()
    a0, a1 = out[0][:, :20], out[1][:, :20]
    scale = np.abs(a1).max(axis=0) + 1e-30
    err = (np.abs(a0 - a1) / scale).max()
    print(f"gate {gate}: max difference {err:.2e} of each term's largest magnitude", flush=True)
    assert err <= 1e-4
    np.testing.assert_array_equal(out[0][:, 20:23], out[1][:, 20:23])     # group centres


def test_captured_correction_and_force_replay_matches_eager(env):
    """The learned correction and the force captured together in one graph (a
    per-step force launch) give bitwise the eager results on every replay,
    with eager work on the same stream between replays."""
    ctx, net, d = env["ctx"], env["net"], env["d"]
    net.set_params(env["params"])
    net.set_gate(0.4)
    try:
        gc = torch.empty((d.n_groups, otoo.CORR_STRIDE), dtype=torch.float32, device="cuda:0")
        out = ctx.outputs(d.n)

        def step():
            ctx.correction(d, otoo.CORR_MLP, EPS, net=net, out=gc)
            ctx.force(d, EPS, out=out, gcorr=gc)

        step()
        torch.cuda.synchronize()
        ref = (out[0].clone(), out[1].clone())
        g = ctx.capture(step)
        for rep in range(3):
            out[0].zero_()
            out[1].zero_()
            gc.zero_()
            ctx.force(d, EPS)                    # eager work between replays
            g.replay()
            torch.cuda.synchronize()
            assert torch.equal(out[0], ref[0]) and torch.equal(out[1], ref[1]), f"replay {rep}"
        ctx.check()
    finally:
        net.set_gate(0.0)
