"""CPU emulator of the force schedule and its reduction structure.

Test infrastructure (NumPy, no GPU).  It models what the library documents
for ``otoo_force``:
- work items (group g, chunk k): a list of length len is one item if
  len <= C, else ceil(len / C) items of C consecutive entries;
- a longest-first order by cost class floor(log2(n_g * item length)), with
  the order inside a class left to the device;
- partial rows for the groups split into several items, in group order;
- the FP32 arithmetic of one item: lanes (target, slice); S = 256 // n_g
  slices of every target, or, where that idles more lanes, up to four wave
  parts of n targets with 64 // n slices each (``lane_parts``); tiles of
  ``tile`` entries, each split into a target's S contiguous runs of
  ceil(len / S) entries (made odd where one wave reads several slices)
  padded with zero-mass entries, a per-tile FP32 sum
  per lane added with Kahan compensation across tiles, the slices combined in
  slice order;
- the merge of a split group's rows in item order (FP32 Kahan for the
  acceleration, FP64 for the potential) and the removal of the self pair.

It is used to check the schedule's capacity bounds, its independence of the
order in which items are processed, and the error behaviour of the
compensated sums, without a GPU.  It shares no code with the library and
calls nothing in it.
"""
from __future__ import annotations

import numpy as np

F32 = np.float32
F64 = np.float64
BLOCK = 256          # threads per workgroup = largest group
CLASSES = 40         # longest-first cost classes


def n_chunks(length: int, chunk: int) -> int:
    return 1 if length <= chunk else -(-length // chunk)


def make_items(list_off, chunk):
    """Items (g, k) in table order: groups ascending, chunks ascending."""
    items = []
    for g in range(len(list_off) - 1):
        for k in range(n_chunks(int(list_off[g + 1] - list_off[g]), chunk)):
            items.append((g, k))
    return items


def item_range(list_off, g, k, chunk):
    lb, le = int(list_off[g]), int(list_off[g + 1])
    cb = lb + k * chunk
    return cb, min(cb + chunk, le)


def cost_class(cost: int) -> int:
    c = int(cost).bit_length() - 1 if cost > 0 else 0
    return min(c, CLASSES - 1)


def lpt_order(items, list_off, group_off, chunk, rng=None):
    """Item indices by cost class, most expensive first.  The device orders
    items inside a class by atomics; ``rng`` draws one such order."""
    by_class = [[] for _ in range(CLASSES)]
    for q, (g, k) in enumerate(items):
        cb, ce = item_range(list_off, g, k, chunk)
        ng = int(group_off[g + 1] - group_off[g])
        by_class[cost_class(ng * max(ce - cb, 1))].append(q)
    order = []
    for c in range(CLASSES - 1, -1, -1):
        members = by_class[c]
        if rng is not None:
            members = list(rng.permutation(members))
        order.extend(members)
    return order


def part_rows(list_off, group_off, chunk):
    """First partial row of every split group (-1 for a group that is one
    item) and the number of rows."""
    base = np.full(len(group_off) - 1, -1, np.int64)
    rows = 0
    for g in range(len(group_off) - 1):
        c = n_chunks(int(list_off[g + 1] - list_off[g]), chunk)
        if c > 1:
            base[g] = rows
            rows += c * int(group_off[g + 1] - group_off[g])
    return base, rows


def _fma(a, b, c):
    # a * b is exact in FP64 for FP32 operands; one rounding to FP32 after the add
    return (a.astype(F64) * b.astype(F64) + c.astype(F64)).astype(F32)


def _kahan(s, c, x):
    y = (x + c).astype(F32)
    t = (s + y).astype(F32)
    c = (y - (t - s)).astype(F32)
    return t, c


def _rsq(x):
    return (1.0 / np.sqrt(x.astype(F64))).astype(F32)


def wave_parts(ng: int):
    """The four wave parts (first target, count) of a group of ng targets that
    does not divide the workgroup, in the documented rule: the largest part
    holds c = 64 // (64 // ceil(ng / 4)) targets; as many parts as fit take c,
    the rest goes to the remaining parts as the largest count 64 // S that
    fits, and the last part takes what is left."""
    c = 64 // (64 // -(-ng // 4))
    nfull = ng // c
    rest = ng - nfull * c
    counts = [c] * nfull
    for j in range(nfull, 4):
        if j == 3:
            take = rest
        else:
            take = 64 // (64 // (rest + 1) + 1) if rest > 0 else 0
        counts.append(take)
        rest -= take
    firsts = np.concatenate([[0], np.cumsum(counts)[:-1]])
    return [(int(b), int(n)) for b, n in zip(firsts, counts)]


def lane_parts(ng: int, tile: int):
    """(targets, S) per part.  Workgroup-wide: all ng targets with
    S = 256 // ng slices, the waves whose lanes all lie past S ng idle; used
    when ng divides 256, or when it runs no more wave rows per full tile than
    the wave parts (and has at most 64 slices).
    Else the wave parts, n targets with 64 // n slices each."""
    S = BLOCK // ng
    parts = [(np.arange(b, b + n), 64 // n) for b, n in wave_parts(ng) if n > 0]
    if BLOCK % ng == 0:
        return [(np.arange(ng), S)]
    part_rows = sum(-(-tile // Sp) for _, Sp in parts)
    shared_rows = -(-(S * ng) // 64) * -(-tile // S)
    if S <= 64 and shared_rows <= part_rows:
        return [(np.arange(ng), S)]
    return parts


def slice_rows(tl: int, S: int, skew: bool) -> int:
    """Rows of each of S slices covering tl entries; odd where one wave reads
    several slices (their LDS records then start in different banks)."""
    rows = -(-tl // S)
    return rows | 1 if skew else rows


def _part_sums(src, xi, idx, eps2, tile, S, skew):
    ng = xi.shape[0]
    s_acc = np.zeros((S, ng, 4), F32)
    c_acc = np.zeros((S, ng, 4), F32)
    for tb in range(0, len(idx), tile):
        tl = min(len(idx) - tb, tile)
        rows = slice_rows(tl, S, skew)
        run = np.zeros((S * rows, 4), F32)      # zero-mass padding
        run[:tl] = src[idx[tb:tb + tl]]
        run = run.reshape(S, rows, 4)            # slice s: entries s*rows .. (s+1)*rows - 1
        part = np.zeros((S, ng, 4), F32)
        for m in range(rows):
            s4 = run[:, m, :]
            dx = (s4[:, None, 0] - xi[None, :, 0]).astype(F32)
            dy = (s4[:, None, 1] - xi[None, :, 1]).astype(F32)
            dz = (s4[:, None, 2] - xi[None, :, 2]).astype(F32)
            r2 = _fma(dx, dx, np.full_like(dx, eps2))
            r2 = _fma(dy, dy, r2)
            r2 = _fma(dz, dz, r2)
            rinv = _rsq(r2)
            mr = (s4[:, None, 3] * rinv).astype(F32)
            mr3 = ((mr * rinv).astype(F32) * rinv).astype(F32)
            part[..., 0] = _fma(mr3, dx, part[..., 0])
            part[..., 1] = _fma(mr3, dy, part[..., 1])
            part[..., 2] = _fma(mr3, dz, part[..., 2])
            part[..., 3] = (part[..., 3] + mr).astype(F32)
        s_acc, c_acc = _kahan(s_acc, c_acc, part)
    s, c = s_acc[0], c_acc[0]
    for sl in range(1, S):
        s, c = _kahan(s, c, (s_acc[sl] + c_acc[sl]).astype(F32))
    return s, c


def item_sums(src, xi, idx, eps2, tile):
    """(sum, comp) [n_g, 4] of one item: acc xyz and the potential sum
    Σ m / r, for targets xi [n_g, 3] (FP32) against the entries idx of the
    source table src [*, 4] (FP32 x, y, z, m)."""
    ng = xi.shape[0]
    eps2 = F32(eps2)
    s = np.zeros((ng, 4), F32)
    c = np.zeros((ng, 4), F32)
    parts = lane_parts(ng, tile)
    for tg, S in parts:
        # one wave reads several slices: parts with S > 1, or a workgroup-wide
        # layout whose slices do not end on wave boundaries
        skew = S > 1 if len(parts) > 1 or BLOCK % ng else ng % 64 != 0 and S <= 64
        s[tg], c[tg] = _part_sums(src, xi[tg], idx, eps2, tile, S, skew)
    return s, c


def force(pos32, mass32, group_off, list_off, list_idx, eps, chunk, tile=512, order=None, cell_mom=None):
    """Emulated otoo_force: (acc [n, 3] FP32, pot [n] FP64).  List entries
    j < n are particles, j >= n the monopole cells of ``cell_mom`` [*, >= 4]
    (COM xyz, M).  ``order`` is the processing order of the items (table
    order if None); every item writes only its own outputs or rows."""
    n = len(mass32)
    src = np.concatenate([pos32.astype(F32), mass32.astype(F32)[:, None]], axis=1)
    if cell_mom is not None and len(cell_mom):
        src = np.concatenate([src, np.asarray(cell_mom, F32)[:, :4]], axis=0)
    eps2 = F32(F32(eps) * F32(eps))
    self_term = (mass32.astype(F32) * _rsq(np.array([eps2]))[0]).astype(F32)
    items = make_items(list_off, chunk)
    base, n_rows = part_rows(list_off, group_off, chunk)
    rows_s = np.zeros((n_rows, 4), F32)
    rows_c = np.zeros((n_rows, 4), F32)
    acc = np.zeros((n, 3), F32)
    pot = np.zeros(n, F64)
    for q in (range(len(items)) if order is None else order):
        g, k = items[q]
        g0, g1 = int(group_off[g]), int(group_off[g + 1])
        cb, ce = item_range(list_off, g, k, chunk)
        s, c = item_sums(src, pos32[g0:g1].astype(F32), np.asarray(list_idx[cb:ce]), eps2, tile)
        if n_chunks(int(list_off[g + 1] - list_off[g]), chunk) == 1:
            acc[g0:g1] = (s[:, :3] + c[:, :3]).astype(F32)
            pot[g0:g1] = -(s[:, 3].astype(F64) + c[:, 3].astype(F64)) + self_term[g0:g1].astype(F64)
        else:
            r0 = base[g] + k * (g1 - g0)
            rows_s[r0:r0 + g1 - g0] = s
            rows_c[r0:r0 + g1 - g0] = c
    for g in range(len(group_off) - 1):
        if base[g] < 0:
            continue
        g0, g1 = int(group_off[g]), int(group_off[g + 1])
        ng = g1 - g0
        s = np.zeros((ng, 3), F32)
        c = np.zeros((ng, 3), F32)
        ph = np.zeros(ng, F64)
        for k in range(n_chunks(int(list_off[g + 1] - list_off[g]), chunk)):
            r0 = base[g] + k * ng
            s, c = _kahan(s, c, (rows_s[r0:r0 + ng, :3] + rows_c[r0:r0 + ng, :3]).astype(F32))
            ph += rows_s[r0:r0 + ng, 3].astype(F64) + rows_c[r0:r0 + ng, 3].astype(F64)
        acc[g0:g1] = (s + c).astype(F32)
        pot[g0:g1] = -ph + self_term[g0:g1].astype(F64)
    return acc, pot
