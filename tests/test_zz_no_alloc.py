"""The no-allocation force entry point (otoo_force_noalloc), called through
the C ABI, against otoo_force on the same inputs: two calls in a row on one
context, the second on a smaller input, each bitwise equal to otoo_force
(the same kernels and schedule, with the scratch in the library's fixed
per-GPU array instead of the context's buffer), and both within the
parity bar of the FP64 oracle.  The array keeps the first call's contents
when the second runs."""
import numpy as np
import pytest

import oracle
import synth
import paper_1206_1199_amd as otoo

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _case(n, seed, theta, g_max, eps):
    pos, m = synth.plummer(n, seed=seed)
    tree = otoo.Tree(pos, m, n_crit=16)
    lists = tree.walk(theta=theta, g_max=g_max)
    _, pos32, mass32, cm = tree.export(4)
    d = otoo.DeviceLists.from_host(pos32, mass32, lists, cm, "cuda:0")
    return d, lists, pos32, mass32, cm, eps


def test_noalloc_matches_force_twice_second_smaller():
    ctx = otoo.Context(0)
    # lists longer than the chunk are split into several items: the partial rows and the
    # reduction pass run in the array too
    ctx.set_tuning(chunk=2048, blocks_per_cu=8, lpt=1, tile=512)
    cases = [_case(1 << 17, 21, 0.5, 64, 0.01), _case(1 << 14, 22, 0.6, 32, 0.02)]
    tu = ctx.tuning()
    for d, lists, pos32, mass32, cm, eps in cases:
        need = otoo.force_plan(d.n, d.n_groups, d.n_entries, d.n_cells, tu.chunk, 256 * tu.blocks_per_cu)
        assert need <= otoo.NOALLOC_SCRATCH_BYTES
        print(f"n={d.n} groups={d.n_groups} entries={d.n_entries}: scratch {need} bytes", flush=True)
        a_ref, p_ref = ctx.force(d, eps)
        gen = ctx.scratch_generation()
        acc = torch.full((d.n, 3), float("nan"), dtype=torch.float32, device="cuda:0")
        pot = torch.full((d.n,), float("nan"), dtype=torch.float64, device="cuda:0")
        rc = otoo.lib().otoo_force_noalloc(*ctx._args(d, eps, acc, pot))
        assert rc == otoo.OK, otoo.lib().otoo_last_error(ctx._h)
        torch.cuda.synchronize()
        ctx.check()
        assert ctx.scratch_generation() == gen          # the context allocated nothing
        assert torch.equal(acc, a_ref) and torch.equal(pot, p_ref)
        a64, p64 = oracle.list_force(pos32.astype(np.float64), mass32.astype(np.float64), lists.group_off,
                                     lists.list_off, lists.list_idx, cm[:, :3].astype(np.float64),
                                     cm[:, 3].astype(np.float64), float(np.float32(eps)))
        ea = oracle.rel_err(acc.cpu().numpy().astype(np.float64), a64)
        ep = oracle.rel_err(pot.cpu().numpy(), p64)
        assert np.median(ea) <= 1e-6 and ea.max() <= 1e-4 and np.median(ep) <= 1e-6 and ep.max() <= 1e-4


def test_noalloc_refuses_debug_validation():
    """The optional host validation copies the lists to host memory, so the
    no-allocation entry point refuses it before anything is enqueued."""
    ctx = otoo.Context(0)
    d, _, _, _, _, eps = _case(4096, 23, 0.5, 64, 0.01)
    ctx.set_tuning(debug_validate=1)
    acc, pot = ctx.outputs(d.n)
    assert otoo.lib().otoo_force_noalloc(*ctx._args(d, eps, acc, pot)) == otoo.EINVAL
    assert b"debug validation" in otoo.lib().otoo_last_error(ctx._h)
