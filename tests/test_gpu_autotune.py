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
