"""The library's autotuner (otoo_autotune): every (group choice, schedule)
pair is timed, the reported best is the fastest, the interaction counts are
those of the host walk, and the context comes back as it was (tuning
restored, no stale graph) and still computes forces at the parity bar."""
import numpy as np
import pytest

import oracle
import synth
import paper_1206_1199_amd as otoo

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

SCHEDULES = [dict(chunk=2048, blocks_per_cu=8, lpt=1, tile=256), dict(chunk=512, blocks_per_cu=4, lpt=0, tile=512),
             dict(chunk=1 << 24, blocks_per_cu=2, lpt=1, tile=256)]
CHOICES = [(otoo.GROUP_CHUNK, 32), (otoo.GROUP_CELL, 64), (otoo.GROUP_CHUNK, 128)]


@pytest.fixture(scope="module")
def setup():
    pos, m = synth.plummer(16384, seed=3)
    return otoo.Context(0), otoo.Tree(pos, m, n_crit=16)


def test_sweep_reports_every_pair_and_the_fastest(setup):
    ctx, tree = setup
    ctx.set_tuning(chunk=1024, blocks_per_cu=6, lpt=1, tile=256)
    before = ctx.tuning().as_dict()
    lists = tree.walk(theta=0.5, g_max=64)
    _, pos32, mass32, cm = tree.export(4)
    d = otoo.DeviceLists.from_host(pos32, mass32, lists, cm, "cuda:0")
    out = ctx.outputs(d.n)
    ctx.graph_capture(d, 0.01, out)
    ms, inter, best_choice, best_t, best_ms = ctx.autotune(tree, 0.01, CHOICES, SCHEDULES, reps=3, theta=0.5)
    print("ms per (choice, schedule):\n", ms, flush=True)
    assert ms.shape == (len(CHOICES), len(SCHEDULES))
    assert np.all(np.isfinite(ms)) and np.all(ms > 0)
    gi, si = np.unravel_index(np.argmin(ms), ms.shape)
    assert best_ms == pytest.approx(float(ms[gi, si]), rel=0, abs=0)
    assert best_choice == CHOICES[gi]
    assert {k: getattr(best_t, k) for k in ("chunk", "blocks_per_cu", "lpt", "tile")} == SCHEDULES[si]
    for (mode, g_max), n_int in zip(CHOICES, inter):
        assert n_int == tree.walk(theta=0.5, g_max=g_max, group_mode=mode).interactions
    assert ctx.tuning().as_dict() == before
    with pytest.raises(otoo.OtooError):   # the sweep's graph named freed buffers: it is gone
        ctx.graph_launch()
    acc, pot = ctx.force(d, 0.01)
    torch.cuda.synchronize()
    ctx.check()
    a_ref, p_ref = oracle.list_force(pos32.astype(np.float64), mass32.astype(np.float64), lists.group_off,
                                     lists.list_off, lists.list_idx, cm[:, :3].astype(np.float64),
                                     cm[:, 3].astype(np.float64), float(np.float32(0.01)))
    ea = oracle.rel_err(acc.cpu().numpy().astype(np.float64), a_ref)
    ep = oracle.rel_err(pot.cpu().numpy(), p_ref)
    assert np.median(ea) <= 1e-6 and ea.max() <= 1e-4
    assert np.median(ep) <= 1e-6 and ep.max() <= 1e-4


def test_rejected_schedule_leaves_tuning_unchanged(setup):
    ctx, tree = setup
    ctx.set_tuning(chunk=4096, blocks_per_cu=8, lpt=0, tile=512)
    before = ctx.tuning().as_dict()
    bad = SCHEDULES[:1] + [dict(chunk=2048, blocks_per_cu=8, lpt=1, tile=300)]
    with pytest.raises(otoo.OtooError) as e:
        ctx.autotune(tree, 0.01, CHOICES[:1], bad, reps=1)
    assert e.value.code == otoo.EINVAL and "tile" in str(e.value)
    assert ctx.tuning().as_dict() == before
    with pytest.raises(otoo.OtooError) as e:
        ctx.autotune(tree, 0.01, [(otoo.GROUP_CHUNK, otoo.MAX_GROUP + 1)], SCHEDULES[:1], reps=1)
    assert e.value.code == otoo.EINVAL
    assert ctx.tuning().as_dict() == before


def test_learned_step_tuned_under_an_error_bound(setup):
    """autotune_learned: for each near ratio the fastest schedule of the
    learned step, the step's median error at the sample measured with it
    (against FP64 direct sums of the oracle), and the fastest ratio within the
    bound; a bound no ratio meets gives the most accurate one."""
    from paper_1206_1199_amd import autotune as at
    from paper_1206_1199_amd import learned
    ctx, tree = setup
    before = ctx.tuning().as_dict()
    net = learned.Network(ctx)
    net.set_params(learned.init_params(5))   # untrained: its errors differ between ratios all the same
    net.set_gate(0.0)
    _, pos32, mass32, _ = tree.export(12)
    sample = synth.sample_idx(len(mass32), 512, seed=9)
    a_ref, _ = oracle.direct(pos32.astype(np.float64), mass32.astype(np.float64), float(np.float32(0.01)),
                             tgt=sample)
    # one group choice and schedule: each ratio's step, and so its error, is the same in both sweeps
    grid = {"group": [(otoo.GROUP_CHUNK, 64)], "chunk": [2048], "blocks_per_cu": [8], "lpt": [1], "tile": [256]}
    ratios = (0.4, 0.6)
    best, rows = at.autotune_learned(tree, 0.01, 0.8, ctx, net, sample, a_ref, ratios=ratios, err_target=1.0,
                                     grid=grid, reps=2)
    assert [r["near_ratio"] for r in rows] == list(ratios)
    for r in rows:
        assert r["median_err"] == pytest.approx(
            at.step_median_error(ctx, tree, 0.01, 0.8, r, net, r["near_ratio"], sample, a_ref), rel=1e-6)
    assert best["near_ratio"] == min(rows, key=lambda r: r["ms"])["near_ratio"] and best["err_target"] == 1.0
    strict, _ = at.autotune_learned(tree, 0.01, 0.8, ctx, net, sample, a_ref, ratios=ratios, err_target=0.0,
                                    grid=grid, reps=2)
    assert strict["near_ratio"] == min(rows, key=lambda r: r["median_err"])["near_ratio"]
    assert ctx.tuning().as_dict() == before
