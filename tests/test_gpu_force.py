"""GPU parity: the HIP force path (through the C ABI) against the FP64 oracle.

Both sides see the same FP32 inputs (positions, masses and cell moments as
exported for the device, promoted to FP64 for the oracle) and the same lists.
Bar (FP32 pair arithmetic with Kahan-compensated accumulation, FP64
potential): median relative error <= 1e-6 and maximum <= 1e-4 per particle
for both acceleration and potential.  Integer outputs (lists) are compared
exactly elsewhere; here runs with different schedules must agree bitwise.
"""
import numpy as np
import pytest

import oracle
import synth
import paper_1206_1199_amd as otoo

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

MED_TOL = 1e-6
MAX_TOL = 1e-4


def _setup(pos64, m64, theta, g_max, mode=otoo.GROUP_CHUNK, stride=4):
    t = otoo.Tree(pos64, m64, n_crit=16)
    lists = t.walk(theta=theta, g_max=g_max, group_mode=mode)
    perm, pos32, mass32, cm = t.export(stride)
    d = otoo.DeviceLists.from_host(pos32, mass32, lists, cm, "cuda:0")
    return t, lists, pos32, mass32, cm, d


def _oracle(pos32, mass32, lists, cm, eps, tgt=None):
    return oracle.list_force(pos32.astype(np.float64), mass32.astype(np.float64), lists.group_off,
                             lists.list_off, lists.list_idx, cm[:, :3].astype(np.float64),
                             cm[:, 3].astype(np.float64), float(np.float32(eps)), tgt=tgt)


def _gpu(ctx, d, eps):
    acc, pot = ctx.force(d, eps)
    torch.cuda.synchronize()
    ctx.check()
    return acc.cpu().numpy().astype(np.float64), pot.cpu().numpy()


def _assert_parity(acc, pot, a_ref, p_ref, label):
    ea = oracle.rel_err(acc, a_ref)
    ep = oracle.rel_err(pot, p_ref)
    print(f"{label}: acc median {np.median(ea):.2e} max {ea.max():.2e} | pot median {np.median(ep):.2e} "
          f"max {ep.max():.2e}", flush=True)
    assert np.median(ea) <= MED_TOL and ea.max() <= MAX_TOL
    assert np.median(ep) <= MED_TOL and ep.max() <= MAX_TOL


@pytest.fixture(scope="module")
def ctx():
    return otoo.Context(0)


@pytest.fixture(scope="module")
def plummer16k():
    return synth.plummer(16384, seed=0)


@pytest.mark.parametrize("g_max,mode", [(64, otoo.GROUP_CHUNK), (64, otoo.GROUP_CELL), (256, otoo.GROUP_CHUNK),
                                        (100, otoo.GROUP_CHUNK), (200, otoo.GROUP_CELL), (17, otoo.GROUP_CHUNK)])
def test_plummer16k_all_particles(ctx, plummer16k, g_max, mode):
    pos, m = plummer16k
    t, lists, pos32, mass32, cm, d = _setup(pos, m, 0.5, g_max, mode)
    ctx.set_tuning(chunk=1024, lpt=1)
    acc, pot = _gpu(ctx, d, 0.01)
    a_ref, p_ref = _oracle(pos32, mass32, lists, cm, 0.01)
    _assert_parity(acc, pot, a_ref, p_ref, f"plummer16k g_max={g_max} mode={mode}")


@pytest.mark.parametrize("dist", ["plummer", "uniform"])
def test_absolute_mac_lists(ctx, dist):
    """Lists of the absolute MAC (Eq. 1 with m_limit = 0.05 of the total mass,
    Sec. 2.2 and 3.3) at Delta = 0.01 and 0.001 through the device force,
    against the oracle's list sums over every particle (16k Plummer sphere and
    uniform sphere, eps 0.01); the tree force against direct sums falls with
    Delta (the oracle's list sums give median errors of 9.0e-4 and 4.2e-4 on
    the Plummer sphere, 3.7e-3 and 1.3e-3 on the uniform sphere)."""
    gen = synth.plummer if dist == "plummer" else synth.uniform_sphere
    pos, m = gen(16384, seed=23)
    t = otoo.Tree(pos, m, n_crit=16)
    _, pos32, mass32, cm = t.export(4)
    sample = synth.sample_idx(len(m), 512, seed=24)
    a_dir, _ = oracle.direct(pos32.astype(np.float64), mass32.astype(np.float64), float(np.float32(0.01)), tgt=sample)
    errs = []
    for delta in (0.01, 0.001):
        lists = t.walk(g_max=64, mac=otoo.MAC_ABSOLUTE, delta=delta, m_limit=0.05)
        assert int(lists.pair_off[-1]) > 0        # cells are accepted
        d = otoo.DeviceLists.from_host(pos32, mass32, lists, cm, "cuda:0")
        acc, pot = _gpu(ctx, d, 0.01)
        a_ref, p_ref = _oracle(pos32, mass32, lists, cm, 0.01)
        _assert_parity(acc, pot, a_ref, p_ref, f"absolute MAC {dist} delta {delta}")
        errs.append(np.median(oracle.rel_err(acc[sample], a_dir)))
    print(f"  tree error vs direct sums: median {errs[0]:.2e} (Delta 0.01), {errs[1]:.2e} (Delta 0.001)", flush=True)
    limits = (1.2e-3, 6e-4) if dist == "plummer" else (5e-3, 1.8e-3)
    assert errs[0] < limits[0] and errs[1] < limits[1] and errs[1] < 0.6 * errs[0]


def test_schedules_agree_bitwise(ctx, plummer16k):
    """Item order (longest-first or table order) and the workgroup count do not
    change a single bit; a short chunk (many items per group, partial rows and
    the reduction kernel) still meets the parity bar."""
    pos, m = plummer16k
    t, lists, pos32, mass32, cm, d = _setup(pos, m, 0.5, 64)
    outs = []
    for lpt, bpc in ((1, 8), (0, 8), (1, 2), (0, 16)):
        ctx.set_tuning(chunk=512, lpt=lpt, blocks_per_cu=bpc)
        outs.append(_gpu(ctx, d, 0.01))
    for a, p in outs[1:]:
        assert np.array_equal(a, outs[0][0]) and np.array_equal(p, outs[0][1])
    ctx.set_tuning(chunk=64, lpt=1, blocks_per_cu=8)
    acc, pot = _gpu(ctx, d, 0.01)
    a_ref, p_ref = _oracle(pos32, mass32, lists, cm, 0.01)
    _assert_parity(acc, pot, a_ref, p_ref, "chunk=64")
    ctx.set_tuning(chunk=1024)


def test_graph_replay_matches_eager(ctx, plummer16k):
    pos, m = plummer16k
    t, lists, pos32, mass32, cm, d = _setup(pos, m, 0.5, 64)
    ctx.set_tuning(chunk=256, lpt=1)
    a_e, p_e = _gpu(ctx, d, 0.01)
    out = ctx.outputs(d.n)
    ctx.graph_capture(d, 0.01, out)
    for rep in range(4):
        out[0].fill_(float("nan"))
        out[1].fill_(float("nan"))
        ctx.graph_launch()
        torch.cuda.synchronize()
        # eager work of the program between replays
        _ = (d.pos * 2).sum().item()
        assert np.array_equal(out[0].cpu().numpy().astype(np.float64), a_e), rep
        assert np.array_equal(out[1].cpu().numpy(), p_e), rep
    ctx.set_tuning(chunk=1024)


def test_theta_zero_equals_direct_sum(ctx):
    pos, m = synth.plummer(2000, seed=5)
    t, lists, pos32, mass32, cm, d = _setup(pos, m, 0.0, 64)
    acc, pot = _gpu(ctx, d, 0.01)
    a_ref, p_ref = oracle.direct(pos32.astype(np.float64), mass32.astype(np.float64), float(np.float32(0.01)))
    _assert_parity(acc, pot, a_ref, p_ref, "theta=0 vs direct")


def test_polytrope_pair_and_cube(ctx):
    pos, m, star, centres = synth.polytrope_pair(8192, seed=2)
    t, lists, pos32, mass32, cm, d = _setup(pos, m, 0.6, 64)
    acc, pot = _gpu(ctx, d, 1e-4)
    a_ref, p_ref = _oracle(pos32, mass32, lists, cm, 1e-4)
    _assert_parity(acc, pot, a_ref, p_ref, "polytrope pair eps=1e-4")
    # per particle class: each star, and cores (r < R/4) against envelopes
    perm = t.export(4)[0]
    r = np.linalg.norm(pos - centres[star], axis=1)
    core = r < np.where(star == 0, 0.02, 0.012) / 4
    for name, mask in (("A", star == 0), ("B", star == 1), ("core", core), ("envelope", ~core)):
        sel = mask[perm]
        _assert_parity(acc[sel], pot[sel], a_ref[sel], p_ref[sel], f"polytrope class {name}")
    pos, m = synth.grf_cube(24, seed=4)
    t, lists, pos32, mass32, cm, d = _setup(pos, m, 0.7, 256, otoo.GROUP_CELL)
    acc, pot = _gpu(ctx, d, 1e-3)
    a_ref, p_ref = _oracle(pos32, mass32, lists, cm, 1e-3)
    _assert_parity(acc, pot, a_ref, p_ref, "grf cube")


@pytest.mark.parametrize("tile", [256, 1024])
@pytest.mark.parametrize("n", [1, 2, 3, 65])
def test_tiny_inputs(ctx, n, tile):
    rng = np.random.default_rng(n)
    pos = rng.normal(size=(n, 3))
    m = rng.uniform(0.5, 1.5, n)
    t, lists, pos32, mass32, cm, d = _setup(pos, m, 0.5, 64)
    ctx.set_tuning(tile=tile)
    try:
        acc, pot = _gpu(ctx, d, 0.05)
    finally:
        ctx.set_tuning(tile=256)
    a_ref, p_ref = _oracle(pos32, mass32, lists, cm, 0.05)
    if n == 1:
        assert np.all(acc == 0) and np.all(pot == 0)
        return
    _assert_parity(acc, pot, a_ref, p_ref, f"n={n}")


def _all_group_sizes(seed):
    """Groups of every size 1..256 in shuffled order, each list holding the
    group's own particles, other particles and cells: lengths drawn around
    the tile boundaries and up to about four 512-entry tiles."""
    rng = synth.rng_for(seed)
    sizes = np.arange(1, 257)
    rng.shuffle(sizes)
    group_off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int32)
    n = int(group_off[-1])
    pos, m = synth.plummer(n, seed=seed)
    pos32, mass32 = pos.astype(np.float32), m.astype(np.float32)
    n_cells = 700
    com = pos32[rng.integers(0, n, n_cells)] + rng.normal(0, 0.05, (n_cells, 3)).astype(np.float32)
    cm = np.concatenate([com, rng.uniform(1e-4, 1e-2, (n_cells, 1))], axis=1).astype(np.float32)
    special = np.array([0, 1, 63, 255, 256, 257, 511, 512, 513, 1023, 1024, 1025, 1536])
    lists, offs = [], [0]
    for g in range(256):
        g0, g1 = int(group_off[g]), int(group_off[g + 1])
        extra = int(special[rng.integers(0, len(special))]) if g % 2 else int(rng.integers(0, 2100))
        n_cell = int(rng.integers(0, extra + 1))
        others = rng.choice(np.concatenate([np.arange(0, g0), np.arange(g1, n)]), extra - n_cell, replace=False)
        idx = np.concatenate([n + rng.choice(n_cells, n_cell), np.arange(g0, g1), others]).astype(np.int32)
        lists.append(idx)
        offs.append(offs[-1] + len(idx))
    return pos32, mass32, cm, group_off, np.array(offs, np.int64), np.concatenate(lists)


@pytest.mark.parametrize("tile,chunk", [(256, 1 << 20), (512, 1 << 20), (1024, 1 << 20), (512, 300)])
def test_every_group_size(ctx, tile, chunk):
    """Every group size 1..256: sizes that divide the workgroup spread each
    target's slices over all its threads, the others mostly take per-wave
    parts of the targets (each part with its own slice count, the parts
    rotating over the waves from item to item); ragged last tiles, empty
    slices and (chunk 300) lists split into several items all meet the bar."""
    pos32, mass32, cm, group_off, list_off, list_idx = _all_group_sizes(41)
    dev = lambda a, dt: torch.from_numpy(np.ascontiguousarray(a, dtype=dt)).to("cuda:0")
    G = len(group_off) - 1
    ng = np.diff(group_off).astype(np.int64)
    d = otoo.DeviceLists(pos=dev(pos32, np.float32), mass=dev(mass32, np.float32),
                         group_off=dev(group_off, np.int32), list_off=dev(list_off, np.int64),
                         list_idx=dev(list_idx, np.int32), cell_mom=dev(cm, np.float32),
                         pair_off=dev(np.zeros(G + 1), np.int64), n_entries=int(list_off[-1]),
                         interactions=int((ng * np.diff(list_off)).sum()), pair_count=0)
    ctx.set_tuning(chunk=chunk, tile=tile, lpt=1)
    try:
        acc, pot = _gpu(ctx, d, 0.01)
    finally:
        ctx.set_tuning(chunk=1024, tile=256)
    a_ref, p_ref = oracle.list_force(pos32.astype(np.float64), mass32.astype(np.float64), group_off, list_off,
                                     list_idx, cm[:, :3].astype(np.float64), cm[:, 3].astype(np.float64),
                                     float(np.float32(0.01)))
    _assert_parity(acc, pot, a_ref, p_ref, f"every group size, tile {tile} chunk {chunk}")


def test_malformed_lists_are_reported(ctx):
    pos, m = synth.plummer(1000, seed=6)
    t, lists, pos32, mass32, cm, d = _setup(pos, m, 0.5, 64)
    bad = d.list_idx.clone()
    bad[5] = d.n + d.n_cells + 7          # out of range: skipped by the kernel, flagged
    d_bad = otoo.DeviceLists(d.pos, d.mass, d.group_off, d.list_off, bad, d.cell_mom, d.pair_off, d.n_entries,
                             d.interactions)
    ctx.force(d_bad, 0.01)
    with pytest.raises(otoo.OtooError):
        ctx.check()
    ctx.check()                            # flag cleared
    ctx.set_tuning(debug_validate=1)
    with pytest.raises(otoo.OtooError):
        ctx.force(d_bad, 0.01)
    ctx.set_tuning(debug_validate=0)
    with pytest.raises(otoo.OtooError):
        ctx.force(d, 0.0)                  # eps must be positive


def test_plummer_1m_sampled(ctx):
    """The benchmark workload (Plummer 2^20, eps 0.005, theta 0.5) on a
    4096-particle sample, in the launch configuration the benchmark times
    (group size and schedule from the autotuner's cache, else its defaults)."""
    from paper_1206_1199_amd import autotune as at
    sched, source = at.cached_schedule("plummer1m")
    mode = otoo.GROUP_CHUNK if sched["group_mode"] == "chunk" else otoo.GROUP_CELL
    pos, m = synth.plummer(1 << 20, seed=1)
    t, lists, pos32, mass32, cm, d = _setup(pos, m, 0.5, sched["g_max"], mode)
    old = ctx.tuning()
    at.apply_schedule(ctx, sched)
    try:
        acc, pot = _gpu(ctx, d, 0.005)
    finally:
        ctx.set_tuning(chunk=old.chunk, blocks_per_cu=old.blocks_per_cu, lpt=old.lpt, tile=old.tile)
    sample = synth.sample_idx(len(m), 4096, seed=101)
    a_ref, p_ref = _oracle(pos32, mass32, lists, cm, 0.005, tgt=sample)
    _assert_parity(acc[sample], pot[sample], a_ref, p_ref, f"plummer 2^20 sample ({source}: {sched})")


def _direct(ctx, pos32, mass32, tgt, eps):
    dev = "cuda:0"
    a, p = ctx.direct(torch.from_numpy(pos32).to(dev), torch.from_numpy(mass32).to(dev),
                      torch.from_numpy(np.asarray(tgt, np.int32)).to(dev), eps)
    torch.cuda.synchronize()
    ctx.check()
    return a.cpu().numpy(), p.cpu().numpy()


def test_direct_sum_matches_oracle(ctx):
    """FP64 direct sums on the device (the accuracy reference of the tree
    force) against the oracle's direct sum: both FP64, different order."""
    pos, m = synth.plummer(20000, seed=8)
    pos32, mass32 = pos.astype(np.float32), m.astype(np.float32)
    tgt = synth.sample_idx(len(m), 999, seed=9)
    a, p = _direct(ctx, pos32, mass32, tgt, 0.01)
    a_ref, p_ref = oracle.direct(pos32.astype(np.float64), mass32.astype(np.float64), float(np.float32(0.01)),
                                 tgt=tgt)
    ea, ep = oracle.rel_err(a, a_ref), oracle.rel_err(p, p_ref)
    print(f"direct: acc max {ea.max():.2e} pot max {ep.max():.2e}", flush=True)
    assert ea.max() <= 1e-12 and ep.max() <= 1e-12
    # a repeated call is bitwise identical
    a2, p2 = _direct(ctx, pos32, mass32, tgt, 0.01)
    assert np.array_equal(a, a2) and np.array_equal(p, p2)


def test_direct_sum_edge_cases(ctx):
    pos32 = np.array([[0, 0, 0], [1, 0, 0], [0, 2, 0]], np.float32)
    mass32 = np.array([1, 2, 3], np.float32)
    a, p = _direct(ctx, pos32[:1], mass32[:1], [0], 0.5)          # one particle: no pair
    assert np.all(a == 0) and np.all(p == 0)
    a, p = _direct(ctx, pos32, mass32, [0, 2, 0], 0.5)            # repeated targets, ragged block
    a_ref, p_ref = oracle.direct(pos32.astype(np.float64), mass32.astype(np.float64), 0.5, tgt=[0, 2, 0])
    assert np.allclose(a, a_ref, rtol=1e-14, atol=0) and np.allclose(p, p_ref, rtol=1e-14, atol=0)
    a, p = _direct(ctx, pos32, mass32, [], 0.5)                   # no targets
    assert a.shape == (0, 3) and p.shape == (0,)
    dev = "cuda:0"
    a_t, p_t = ctx.direct(torch.from_numpy(pos32).to(dev), torch.from_numpy(mass32).to(dev),
                          torch.tensor([1, 3], dtype=torch.int32, device=dev), 0.5)   # index 3 is out of range
    torch.cuda.synchronize()
    with pytest.raises(otoo.OtooError):
        ctx.check()
    assert np.all(a_t.cpu().numpy()[1] == 0)
    with pytest.raises(otoo.OtooError):
        ctx.direct(torch.from_numpy(pos32).to(dev), torch.from_numpy(mass32).to(dev),
                   torch.tensor([0], dtype=torch.int32, device=dev), 0.0)


def _oracle_quad(pos32, mass32, lists, cm, eps, quad, tgt=None):
    return oracle.list_force(pos32.astype(np.float64), mass32.astype(np.float64), lists.group_off,
                             lists.list_off, lists.list_idx, cm[:, :3].astype(np.float64),
                             cm[:, 3].astype(np.float64), float(np.float32(eps)), tgt=tgt,
                             n_cellent=lists.n_cellent, quad=quad, expanded=True)


def test_cell_tensors_local_expansion(ctx, plummer16k):
    """Random per-(group, cell) tensors applied through the group local
    expansion: same bar as the monopole path (the expansion is FP32, the
    correction it carries is small)."""
    pos, m = plummer16k
    t, lists, pos32, mass32, cm, d = _setup(pos, m, 0.7, 64, stride=12)
    n_pairs = int(lists.pair_off[-1])
    rng = np.random.default_rng(21)
    scale = (cm[:, 3] * cm[:, 4] ** 2)[lists.list_idx[np.concatenate(
        [np.arange(lists.list_off[g], lists.list_off[g] + lists.n_cellent[g]) for g in range(lists.n_groups)])]
        - t.n]
    quad = (rng.normal(size=(n_pairs, 6)) * 0.3 * scale[:, None]).astype(np.float32)
    corr = torch.from_numpy(quad).cuda()
    gc = ctx.correction(d, otoo.CORR_PAIRS, 0.01, corr=corr)
    acc, pot = ctx.force(d, 0.01, gcorr=gc)
    torch.cuda.synchronize()
    ctx.check()
    a_ref, p_ref = _oracle_quad(pos32, mass32, lists, cm, 0.01, quad.astype(np.float64))
    _assert_parity(acc.cpu().numpy().astype(np.float64), pot.cpu().numpy(), a_ref, p_ref, "random cell tensors")


def test_exact_quadrupole_pairs_and_accuracy(ctx, plummer16k):
    """Device quadrupole tensors equal 3S - tr(S) I of the exported cell
    moments (FP32, 1e-6 relative); the fused quadrupole correction meets the
    parity bar; at theta = 0.8 it beats the plain monopole against the direct
    sum."""
    from oracle import mlp as omlp
    pos, m = plummer16k
    t, lists, pos32, mass32, cm, d = _setup(pos, m, 0.8, 64, stride=12)
    corr = ctx.quad_exact(d)
    torch.cuda.synchronize()
    ctx.check()
    cells = np.concatenate([lists.list_idx[lists.list_off[g]:lists.list_off[g] + lists.n_cellent[g]]
                            for g in range(lists.n_groups)]) - t.n
    q_ref = omlp.exact_quadrupole(cm[cells, 5:11].astype(np.float64))
    q_gpu = corr.cpu().numpy().astype(np.float64)
    np.testing.assert_allclose(q_gpu, q_ref, rtol=1e-6, atol=1e-6 * np.abs(q_ref).max())
    gc = ctx.correction(d, otoo.CORR_QUAD, 0.01)
    acc, pot = ctx.force(d, 0.01, gcorr=gc)
    torch.cuda.synchronize()
    ctx.check()
    a_q = acc.cpu().numpy().astype(np.float64)
    a_ref, p_ref = _oracle_quad(pos32, mass32, lists, cm, 0.01, q_ref)
    _assert_parity(a_q, pot.cpu().numpy(), a_ref, p_ref, "exact quadrupole")
    a_m, _ = _gpu(ctx, d, 0.01)
    sample = synth.sample_idx(len(m), 1024, seed=100)
    a_dir, _ = oracle.direct(pos32.astype(np.float64), mass32.astype(np.float64), float(np.float32(0.01)),
                             tgt=sample)
    e_q = np.median(oracle.rel_err(a_q[sample], a_dir))
    e_m = np.median(oracle.rel_err(a_m[sample], a_dir))
    print(f"theta 0.8: monopole median {e_m:.2e}, with quadrupole {e_q:.2e}", flush=True)
    assert e_q < 0.75 * e_m


@pytest.mark.parametrize("tile", [512, 1024])
@pytest.mark.parametrize("g_max", [32, 64, 256])
def test_deeper_tiles(ctx, plummer16k, g_max, tile):
    # chunk 1536: lists split into items with ragged last tiles
    pos, m = plummer16k
    t, lists, pos32, mass32, cm, d = _setup(pos, m, 0.5, g_max)
    ctx.set_tuning(chunk=1536, tile=tile, lpt=1)
    acc, pot = _gpu(ctx, d, 0.01)
    ctx.set_tuning(chunk=1024, tile=256)
    a_ref, p_ref = _oracle(pos32, mass32, lists, cm, 0.01)
    _assert_parity(acc, pot, a_ref, p_ref, f"tile {tile} g_max={g_max}")


@pytest.mark.parametrize("workload", ["polytrope2m", "cube16m"])
def test_full_size_workloads_sampled(ctx, workload):
    """The two-polytrope (2 x 2^20) and GRF-cube (2^24) workloads at full size,
    in the launch configuration the benchmark times for them (autotuner cache
    or defaults), against the oracle's list sums on 2048 sampled particles."""
    from paper_1206_1199_amd import autotune as at
    if workload == "polytrope2m":
        pos, m, _, _ = synth.polytrope_pair(1 << 20, seed=2)
        eps, theta, seed = 1e-4, 0.6, 102
    else:
        pos, m = synth.grf_cube(256, seed=4)
        eps, theta, seed = 1e-3, 0.7, 104
    sched, source = at.cached_schedule(workload)
    mode = otoo.GROUP_CHUNK if sched["group_mode"] == "chunk" else otoo.GROUP_CELL
    t, lists, pos32, mass32, cm, d = _setup(pos, m, theta, sched["g_max"], mode)
    old = ctx.tuning()
    at.apply_schedule(ctx, sched)
    try:
        acc, pot = _gpu(ctx, d, eps)
    finally:
        ctx.set_tuning(chunk=old.chunk, blocks_per_cu=old.blocks_per_cu, lpt=old.lpt, tile=old.tile)
    sample = synth.sample_idx(len(m), 2048, seed=seed)
    a_ref, p_ref = _oracle(pos32, mass32, lists, cm, eps, tgt=sample)
    _assert_parity(acc[sample], pot[sample], a_ref, p_ref, f"{workload} sample ({source}: {sched})")


def test_corrections_split_into_segments(ctx):
    """Groups with more cell pairs than one segment (1024) are summed by
    several waves and their segment sums merged in segment order; groups
    with fewer take one wave.  The textbook quadrupole through both kinds of
    item meets the parity bar, and a second call gives the same bits."""
    from oracle import mlp as omlp
    pos, m = synth.plummer(32768, seed=6)
    t, lists, pos32, mass32, cm, d = _setup(pos, m, 0.25, 256, stride=12)
    nce = np.asarray(lists.n_cellent)
    assert (nce > 2 * 1024).any() and (nce <= 1024).any()
    gc = ctx.correction(d, otoo.CORR_QUAD, 0.01)
    acc, pot = ctx.force(d, 0.01, gcorr=gc)
    torch.cuda.synchronize()
    ctx.check()
    cells = np.concatenate([lists.list_idx[lists.list_off[g]:lists.list_off[g] + lists.n_cellent[g]]
                            for g in range(lists.n_groups)]) - t.n
    q_ref = omlp.exact_quadrupole(cm[cells, 5:11].astype(np.float64))
    sample = synth.sample_idx(len(m), 4096, seed=7)
    a_ref, p_ref = _oracle_quad(pos32, mass32, lists, cm, 0.01, q_ref, tgt=sample)
    _assert_parity(acc.cpu().numpy().astype(np.float64)[sample], pot.cpu().numpy()[sample], a_ref, p_ref,
                   "quadrupole, split groups")
    gc2 = ctx.correction(d, otoo.CORR_QUAD, 0.01)
    torch.cuda.synchronize()
    assert torch.equal(gc, gc2)


def test_captured_graph_dropped_when_scratch_grows():
    """A graph captured on a context names its scratch; a later call that
    grows the scratch discards the graph, so replaying it fails cleanly
    instead of touching freed memory.  A new capture works again."""
    c = otoo.Context(0)
    pos, m = synth.plummer(2000, seed=8)
    _, _, _, _, _, d_small = _setup(pos, m, 0.5, 64)
    out = c.outputs(d_small.n)
    c.graph_capture(d_small, 0.01, out)
    c.graph_launch()
    torch.cuda.synchronize()
    pos, m = synth.plummer(16384, seed=9)
    _, lists, pos32, mass32, cm, d_big = _setup(pos, m, 0.5, 64)
    acc, pot = _gpu(c, d_big, 0.01)
    with pytest.raises(otoo.OtooError) as e:
        c.graph_launch()
    assert e.value.code == otoo.EINVAL
    out_big = c.outputs(d_big.n)
    c.graph_capture(d_big, 0.01, out_big)
    c.graph_launch()
    torch.cuda.synchronize()
    assert np.array_equal(out_big[0].cpu().numpy().astype(np.float64), acc)


def test_captured_step_refuses_replay_after_scratch_grows():
    """A torch graph of library calls (Context.capture) names the context's
    scratch of the moment.  A later eager call that needs more scratch makes
    the context allocate anew; the captured step then refuses to replay (it
    would write freed memory) without being replayed, and a new capture
    gives the eager result again."""
    c = otoo.Context(0)
    pos, m = synth.plummer(2000, seed=8)
    d_small = _setup(pos, m, 0.5, 64, stride=12)[-1]
    out = c.outputs(d_small.n)
    gc = torch.empty((d_small.n_groups, otoo.CORR_STRIDE), dtype=torch.float32, device="cuda:0")

    def step():
        c.correction(d_small, otoo.CORR_QUAD, 0.01, out=gc)
        c.force(d_small, 0.01, out=out, gcorr=gc)

    g = c.capture(step)
    g.replay()
    torch.cuda.synchronize()
    ref = out[0].clone()
    gen = c.scratch_generation()
    assert not g.stale()
    pos, m = synth.plummer(16384, seed=9)
    d_big = _setup(pos, m, 0.5, 64, stride=12)[-1]
    gc_big = c.correction(d_big, otoo.CORR_QUAD, 0.01)
    c.force(d_big, 0.01, gcorr=gc_big)
    torch.cuda.synchronize()
    assert c.scratch_generation() > gen
    assert g.stale()
    with pytest.raises(otoo.OtooError) as e:
        g.replay()
    assert e.value.code == otoo.EINVAL
    g2 = c.capture(step)
    out[0].zero_()
    g2.replay()
    torch.cuda.synchronize()
    assert torch.equal(out[0], ref)
    c.check()


def test_correction_without_cells(ctx):
    """theta = 0 opens every cell: no group has cell pairs, so every row of the
    correction is zero terms with the group's box centre (written by the
    merge pass), and the corrected force equals the plain one bit for bit."""
    pos, m = synth.plummer(3000, seed=13)
    t, lists, pos32, mass32, cm, d = _setup(pos, m, 0.0, 64, stride=12)
    assert int(lists.pair_off[-1]) == 0
    gc = ctx.correction(d, otoo.CORR_QUAD, 0.01)
    acc, pot = ctx.force(d, 0.01, gcorr=gc)
    torch.cuda.synchronize()
    ctx.check()
    g = gc.cpu().numpy()
    assert np.all(g[:, :20] == 0) and np.all(g[:, 23] == 0)
    go = np.asarray(lists.group_off)
    centre = np.stack([0.5 * (pos32[go[i]:go[i + 1]].min(0) + pos32[go[i]:go[i + 1]].max(0))
                       for i in range(lists.n_groups)])
    np.testing.assert_allclose(g[:, 20:23], centre, rtol=0, atol=1e-6)
    a0, p0 = _gpu(ctx, d, 0.01)
    assert np.array_equal(acc.cpu().numpy().astype(np.float64), a0) and np.array_equal(pot.cpu().numpy(), p0)


def test_scratch_cap():
    """A scratch cap below what a call needs makes the call fail with ENOMEM
    before it enqueues anything (force, correction and SPH passes); without
    the cap the same calls work on the same context."""
    c = otoo.Context(0)
    pos, m = synth.plummer(4096, seed=14)
    t, lists, pos32, mass32, cm, d = _setup(pos, m, 0.6, 64, stride=12)
    with pytest.raises(otoo.OtooError):
        c.set_scratch_limit(-1)
    c.set_scratch_limit(1024)
    for call in (lambda: c.force(d, 0.01), lambda: c.correction(d, otoo.CORR_QUAD, 0.01)):
        with pytest.raises(otoo.OtooError) as e:
            call()
        assert e.value.code == otoo.ENOMEM and "cap" in str(e.value)
    h = torch.full((d.n,), 0.05, dtype=torch.float32, device="cuda:0")
    sl = t.walk_sph(np.full(len(m), 0.05), g_max=64)
    ds = otoo.DeviceLists.from_host(pos32, mass32, sl, cm, "cuda:0")
    with pytest.raises(otoo.OtooError) as e:
        c.sph_sum(ds, h, ds.mass)
    assert e.value.code == otoo.ENOMEM
    c.set_scratch_limit(0)
    a_cap, p_cap = _gpu(c, d, 0.01)
    a_ref, p_ref = _gpu(otoo.Context(0), d, 0.01)
    assert np.array_equal(a_cap, a_ref) and np.array_equal(p_cap, p_ref)
    c.correction(d, otoo.CORR_QUAD, 0.01)
    c.sph_sum(ds, h, ds.mass)
    torch.cuda.synchronize()
    c.check()
