"""The force schedule checked on the CPU through its emulator (tests/emu_sched.py).

- Work items tile every list exactly once and fit the capacity the library
  reserves: n_groups + floor(n_entries / C) + 1 items, and partial rows for
  at most min(that, 2 floor(n_entries / C) + 1) split items of up to 256
  targets (a split list has len > C, so at most 2 len / C items), and at most
  n (floor(n_entries / C) + 1) rows.
- The longest-first order is a permutation with non-increasing cost class.
- The emulated FP32 sums meet the parity bar against the FP64 oracle for
  every chunk and tile, and do not depend on the order in which items run.
- Compensated tile sums keep a long list's error at the level of a short one,
  where a single running FP32 sum does not.
"""
import numpy as np
import pytest

import emu_sched as emu
import oracle
import synth
import paper_1206_1199_amd as otoo

MED_TOL = 1e-6
MAX_TOL = 1e-4


def _lengths(rng, n_groups, chunk):
    # adversarial lengths around the chunk boundaries mixed with a heavy tail
    special = np.array([1, 2, chunk - 1, chunk, chunk + 1, 2 * chunk, 2 * chunk + 1, 3 * chunk - 1, 7 * chunk + 3])
    pick = rng.integers(0, 3, n_groups)
    tail = np.maximum(1, rng.lognormal(np.log(chunk), 1.5, n_groups).astype(np.int64))
    return np.where(pick == 0, special[rng.integers(0, len(special), n_groups)], tail)


@pytest.mark.parametrize("seed", range(6))
@pytest.mark.parametrize("chunk", [64, 1000, 4096])
def test_items_cover_each_list_once_within_reserved_capacity(seed, chunk):
    rng = synth.rng_for(100 + seed)
    n_groups = int(rng.integers(1, 400))
    lens = _lengths(rng, n_groups, chunk)
    list_off = np.concatenate([[0], np.cumsum(lens)])
    sizes = rng.integers(1, 257, n_groups) if seed % 2 else np.full(n_groups, 256)
    group_off = np.concatenate([[0], np.cumsum(sizes)])
    n, n_entries = int(group_off[-1]), int(list_off[-1])

    items = emu.make_items(list_off, chunk)
    covered = np.zeros(n_entries, np.int64)
    last = {}
    for g, k in items:
        cb, ce = emu.item_range(list_off, g, k, chunk)
        assert list_off[g] <= cb and ce <= list_off[g + 1]
        assert k == last.get(g, -1) + 1      # chunks of a group are consecutive
        last[g] = k
        covered[cb:ce] += 1
    assert np.all(covered == 1)
    assert len(last) == n_groups             # every group has an item, empty or not

    item_cap = n_groups + n_entries // chunk + 1
    assert len(items) <= item_cap
    split_items = min(item_cap, 2 * (n_entries // chunk) + 1)
    part_cap = max(1, min(split_items * 256, n * (n_entries // chunk + 1)))
    _, rows = emu.part_rows(list_off, group_off, chunk)
    assert rows <= part_cap


def test_longest_first_order_is_a_permutation_by_class():
    rng = synth.rng_for(7)
    chunk = 512
    lens = _lengths(rng, 300, chunk)
    list_off = np.concatenate([[0], np.cumsum(lens)])
    group_off = np.concatenate([[0], np.cumsum(rng.integers(1, 257, 300))])
    items = emu.make_items(list_off, chunk)
    for r in (None, synth.rng_for(8)):
        order = emu.lpt_order(items, list_off, group_off, chunk, rng=r)
        assert sorted(order) == list(range(len(items)))
        cls = []
        for q in order:
            g, k = items[q]
            cb, ce = emu.item_range(list_off, g, k, chunk)
            cls.append(emu.cost_class(int(group_off[g + 1] - group_off[g]) * max(ce - cb, 1)))
        assert all(a >= b for a, b in zip(cls, cls[1:]))


@pytest.fixture(scope="module")
def plummer4k():
    pos, m = synth.plummer(4096, 5)
    t = otoo.Tree(pos, m, n_crit=16)
    lists = t.walk(theta=0.5, g_max=64)
    _, p32, m32, cm = t.export(4)
    eps = 0.01
    ref = oracle.list_force(p32.astype(np.float64), m32.astype(np.float64), lists.group_off, lists.list_off,
                            lists.list_idx, cm[:, :3].astype(np.float64), cm[:, 3].astype(np.float64),
                            float(np.float32(eps)))
    return p32, m32, cm, lists, eps, ref


@pytest.mark.parametrize("chunk,tile", [(1 << 20, 512), (256, 512), (64, 256)])
def test_emulated_schedule_meets_parity_bar(plummer4k, chunk, tile):
    p32, m32, cm, L, eps, (a_ref, p_ref) = plummer4k
    acc, pot = emu.force(p32, m32, L.group_off, L.list_off, L.list_idx, eps, chunk, tile, cell_mom=cm)
    ea, ep = oracle.rel_err(acc, a_ref), oracle.rel_err(pot, p_ref)
    assert np.median(ea) <= MED_TOL and ea.max() <= MAX_TOL
    assert np.median(ep) <= MED_TOL and ep.max() <= MAX_TOL


def test_emulated_wave_parts_meet_parity_bar():
    """Cell groups of many sizes (wave parts with their odd rows, and
    workgroup-wide layouts) meet the bar."""
    pos, m = synth.plummer(3000, 8)
    t = otoo.Tree(pos, m, n_crit=16)
    L = t.walk(theta=0.6, g_max=100, group_mode=otoo.GROUP_CELL)
    _, p32, m32, cm = t.export(4)
    sizes = np.diff(L.group_off)
    assert any(len(emu.lane_parts(int(g), 512)) > 1 for g in sizes)
    eps = 0.01
    a_ref, p_ref = oracle.list_force(p32.astype(np.float64), m32.astype(np.float64), L.group_off, L.list_off,
                                     L.list_idx, cm[:, :3].astype(np.float64), cm[:, 3].astype(np.float64),
                                     float(np.float32(eps)))
    acc, pot = emu.force(p32, m32, L.group_off, L.list_off, L.list_idx, eps, 1 << 20, 512, cell_mom=cm)
    ea, ep = oracle.rel_err(acc, a_ref), oracle.rel_err(pot, p_ref)
    assert np.median(ea) <= MED_TOL and ea.max() <= MAX_TOL
    assert np.median(ep) <= MED_TOL and ep.max() <= MAX_TOL


def test_processing_order_does_not_change_results(plummer4k):
    p32, m32, cm, L, eps, _ = plummer4k
    chunk = 256
    items = emu.make_items(L.list_off, chunk)
    assert len(items) > L.n_groups   # some lists are split
    orders = [None, emu.lpt_order(items, L.list_off, L.group_off, chunk),
              emu.lpt_order(items, L.list_off, L.group_off, chunk, rng=synth.rng_for(3)),
              list(range(len(items)))[::-1]]
    runs = [emu.force(p32, m32, L.group_off, L.list_off, L.list_idx, eps, chunk, 512, order=o, cell_mom=cm)
            for o in orders]
    for acc, pot in runs[1:]:
        assert np.array_equal(acc, runs[0][0]) and np.array_equal(pot, runs[0][1])


def test_compensated_tiles_keep_long_lists_accurate():
    # 64 targets near the origin, 2^16 sources in a shell at distance 2-4
    rng = synth.rng_for(11)
    ns = 1 << 16
    tgt = rng.uniform(-0.02, 0.02, (64, 3))
    d = rng.normal(size=(ns, 3))
    d /= np.linalg.norm(d, axis=1)[:, None]
    src = d * rng.uniform(2.0, 4.0, ns)[:, None] + np.array([0.5, 0.0, 0.0])
    pos = np.concatenate([tgt, src]).astype(np.float32)
    mass = np.full(len(pos), 1.0 / len(pos), np.float32)
    go, lo, li = np.array([0, 64]), np.array([0, len(pos)]), np.arange(len(pos), dtype=np.int32)
    eps = 0.01
    a_ref, p_ref = oracle.list_force(pos.astype(np.float64), mass.astype(np.float64), go, lo, li,
                                     np.zeros((0, 3)), np.zeros(0), float(np.float32(eps)), tgt=np.arange(64))
    acc, pot = emu.force(pos, mass, go, lo, li, eps, chunk=1 << 30, tile=512)
    ea, ep = oracle.rel_err(acc[:64], a_ref), oracle.rel_err(pot[:64], p_ref)

    # the same pair terms summed in one running FP32 accumulator per target
    x = pos[:64]
    eps2 = np.float32(np.float32(eps) ** 2)
    ax = np.zeros((64, 3), np.float32)
    ph = np.zeros(64, np.float32)
    for j in range(len(pos)):
        dd = (pos[j] - x).astype(np.float32)
        r2 = (np.sum(dd.astype(np.float64) ** 2, axis=1) + eps2).astype(np.float32)
        ri = (1.0 / np.sqrt(r2.astype(np.float64))).astype(np.float32)
        mr = (mass[j] * ri).astype(np.float32)
        ax = (ax + (mr * ri * ri)[:, None] * dd).astype(np.float32)
        ph = (ph + mr).astype(np.float32)
    na = oracle.rel_err(ax, a_ref)
    npot = oracle.rel_err(-ph.astype(np.float64) + mass[:64].astype(np.float64) / np.float32(eps), p_ref)
    print(f"tiles + Kahan: acc {np.median(ea):.2e}, pot {np.median(ep):.2e}; "
          f"one running sum: acc {np.median(na):.2e}, pot {np.median(npot):.2e}")
    assert np.median(ea) <= 5e-7 and np.median(ep) <= 1e-7
    assert np.median(na) >= 10 * np.median(ea) and np.median(npot) >= 10 * np.median(ep)


@pytest.mark.parametrize("tile", [256, 512, 1024])
def test_lane_layout_covers_each_target_and_entry_once(tile):
    """Every group size 1..256: the parts hold each target once, at most 64
    targets a wave part, the slices of a target cover a tile's entries once,
    and the rows a slice reads (odd where several slices share a wave) stay
    within the tile and its 128 zero records.
    The layout chosen never runs more wave rows per full tile than the
    workgroup-wide one, its longest part no more rows than that layout with
    ceil(ng / 4) targets a wave, and from 33 targets on it issues at most
    14 % more rows than ng / 64 per entry."""
    worse = 0
    for ng in range(1, 257):
        parts = emu.lane_parts(ng, tile)
        tg = np.concatenate([p for p, _ in parts])
        assert np.array_equal(np.sort(tg), np.arange(ng))
        if len(parts) > 1 or emu.BLOCK % ng:
            assert len(emu.wave_parts(ng)) == 4
        if len(parts) > 1:
            assert all(len(p) <= 64 and S == 64 // len(p) for p, S in parts)
        for _, S in parts:
            wave_parts_used = len(parts) > 1 or (emu.BLOCK % ng != 0 and S != emu.BLOCK // ng)
            skew = S > 1 if wave_parts_used else ng % 64 != 0 and S <= 64
            assert S <= 64 or not skew
            for tl in (1, tile - 1, tile):
                rows = emu.slice_rows(tl, S, skew)
                assert S * rows >= tl and S * rows <= tile + 128
                cover = np.zeros(S * rows, np.int64)
                for sl in range(S):
                    cover[sl * rows:(sl + 1) * rows] += 1
                assert np.all(cover == 1)
        S0 = emu.BLOCK // ng
        shared = -(-(S0 * ng) // 64) * -(-tile // S0)
        issued = sum(-(-tile // S) * (-(-len(p) * S // 64)) for p, S in parts)
        assert issued <= shared or (S0 > 64 and len(parts) > 1)
        ws = 64 // -(-ng // 4)
        assert max(-(-tile // S) for _, S in parts) <= -(-tile // min(ws, S0))
        if ng >= 33:
            assert issued <= 1.14 * tile * ng / 64, ng
        worse += issued < shared
    assert worse > 100     # most sizes that do not divide 256 gain


def test_small_division_through_the_reciprocal():
    """The force kernel divides lane, slice and row counts (0 <= x <= 2048,
    1 <= d <= 256) as floor((x + 1/2) * rcp(d)) in FP32; exact for a
    reciprocal within one ulp either side of 1 / d."""
    x = np.arange(0, 2049, dtype=np.float32)[:, None]
    d = np.arange(1, 257, dtype=np.float32)[None, :]
    r0 = (np.float32(1.0) / d).astype(np.float32)
    want = np.arange(0, 2049)[:, None] // np.arange(1, 257)[None, :]
    for r in (r0, np.nextafter(r0, np.float32(0)), np.nextafter(r0, np.float32(1))):
        q = np.floor(((x + np.float32(0.5)).astype(np.float32) * r).astype(np.float32)).astype(np.int64)
        assert np.array_equal(q, want)


@pytest.mark.parametrize("tile", [256, 512, 1024])
def test_library_layout_matches_the_model(tile):
    """The layout table compiled into the force kernel (read back through
    otoo_group_layout, host only) gives every group size the layout of the
    model above: the same wave parts, or the same workgroup-wide slices."""
    for ng in range(1, 257):
        wave_parts, parts = otoo.group_layout(ng, tile)
        model = emu.lane_parts(ng, tile)
        model_parts = len(model) > 1 or (emu.BLOCK % ng != 0 and model[0][1] != emu.BLOCK // ng)
        assert wave_parts == model_parts, ng
        if wave_parts:
            assert parts == [n for _, n in emu.wave_parts(ng)], ng
        else:
            assert parts == [emu.BLOCK // ng, 0, 0, 0], ng
    for bad in ((0, tile), (257, tile), (64, 300)):
        with pytest.raises(otoo.OtooError):
            otoo.group_layout(*bad)
