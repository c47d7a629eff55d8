"""Autotuner for the force evaluation: group size and mode (host walk) and the
device schedule (chunk length, workgroups per CU, item order, tile depth).

The objective is the wall time of one full force evaluation (a graph replay
with device-resident inputs) at the workload's opening angle: larger groups
raise the interaction count, so interactions per second alone would favour
them; the time per evaluation is what a simulation pays.  Results are cached
in a JSON file keyed by device architecture, compute-unit count and workload.
"""
from __future__ import annotations

import itertools
import json
import os

from . import CORR_MLP, GROUP_CELL, GROUP_CHUNK, Context, Tree

PACKAGE_CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "autotune_cache.json")


def default_cache(environ=None) -> str:
    """The cache file: OTOO_AUTOTUNE_CACHE if set, else the package's."""
    env = os.environ if environ is None else environ
    return env.get("OTOO_AUTOTUNE_CACHE", "").strip() or PACKAGE_CACHE


DEFAULT_CACHE = default_cache()
TIE = 0.01   # relative time difference below which two schedules count as equally fast

GRID = {
    "group": [(GROUP_CHUNK, 32), (GROUP_CHUNK, 64), (GROUP_CHUNK, 128), (GROUP_CELL, 64), (GROUP_CELL, 128),
              (GROUP_CELL, 256)],
    "chunk": [2048, 4096, 8192, 16384, 1 << 24],
    "blocks_per_cu": [4, 6, 8],
    "lpt": [0, 1],
    "tile": [256, 512, 1024],
}


def device_key(device: int = 0) -> str:
    import torch
    p = torch.cuda.get_device_properties(device)
    arch = getattr(p, "gcnArchName", "unknown").split(":")[0]
    return f"{arch}:{p.multi_processor_count}cu"


def autotune(tree: Tree, eps: float, theta: float, ctx: Context, grid=None, reps: int = 10, log=None,
             corr_kind: int = -1, net=None, near_ratio: float = 0.0):
    """Sweep the grid through the library's otoo_autotune (otoo_autotune_step
    when corr_kind is CORR_QUAD or CORR_MLP: the timed step is the correction
    pass and the force; near_ratio > 0 corrects only the near cells that the
    walk lists first); returns (best dict, table of all measurements).  The
    best is the fastest schedule, or, among those within 1 % of it, the one
    with the most interactions per second."""
    grid = grid or GRID
    choices = list(grid["group"])
    schedules = [dict(chunk=c, blocks_per_cu=b, lpt=l, tile=t)
                 for c, b, l, t in itertools.product(grid["chunk"], grid["blocks_per_cu"], grid["lpt"], grid["tile"])]
    ctx.sync_stream()
    ms, inter, _, _, _ = ctx.autotune(tree, eps, choices, schedules, reps=reps, theta=theta, corr_kind=corr_kind,
                                      net=net, near_ratio=near_ratio)
    table = []
    for gi, (mode, g_max) in enumerate(choices):
        rows = [dict(group_mode="chunk" if mode == GROUP_CHUNK else "cell", g_max=g_max, **s, ms=float(ms[gi, si]),
                     interactions=int(inter[gi]), gint_s=float(inter[gi] / ms[gi, si] / 1e6))
                for si, s in enumerate(schedules)]
        table += rows
        if log:
            b = min(rows, key=lambda r: r["ms"])
            log(f"  {b['group_mode']} g_max={g_max}: best {b['ms']:.3f} ms ({b['gint_s']:.0f} Gint/s)")
    # schedules within TIE of the fastest cost the same within timing noise;
    # among them the one with the highest interaction rate is kept
    fastest = min(r["ms"] for r in table)
    best = max((r for r in table if r["ms"] <= fastest * (1.0 + TIE)), key=lambda r: r["gint_s"])
    return best, table


# near ratios the learned step is tuned over (the network is trained on pairs
# of ratio >= 0.4, so each of these corrects a subset of its training pairs),
# and the median force error the tuned step must hold
NEAR_RATIOS = (0.4, 0.5, 0.55, 0.6, 0.62, 0.65)
ERR_TARGET = 1e-3


def choose_near_ratio(rows, err_target: float = ERR_TARGET):
    """Among rows (one per near ratio: its fastest schedule's "ms" and the
    step's measured "median_err"), the fastest whose error is at most
    err_target; if none is, the most accurate."""
    ok = [r for r in rows if r["median_err"] <= err_target]
    if ok:
        return min(ok, key=lambda r: r["ms"])
    return min(rows, key=lambda r: r["median_err"])


def step_median_error(ctx: Context, tree: Tree, eps: float, theta: float, sched: dict, net, near_ratio: float,
                      sample, a_ref) -> float:
    """Median relative acceleration error, at the particles `sample` (device
    order) against the reference accelerations a_ref [len(sample), 3], of one
    learned step (correction of the near cells, then the force) with the
    given schedule.  Leaves the context's tuning as it was."""
    import numpy as np
    import torch
    from . import CORR_STRIDE
    from .learned import device_tree_arrays
    old = ctx.tuning()
    try:
        apply_schedule(ctx, sched)
        lists = tree.walk(theta=theta, g_max=int(sched["g_max"]),
                          group_mode=GROUP_CHUNK if sched["group_mode"] == "chunk" else GROUP_CELL,
                          near_ratio=near_ratio)
        d, _, _ = device_tree_arrays(tree, lists)
        gc = torch.empty((d.n_groups, CORR_STRIDE), dtype=torch.float32, device=d.pos.device)
        acc, _ = ctx.force(d, eps, gcorr=ctx.correction(d, CORR_MLP, eps, net=net, out=gc))
        torch.cuda.synchronize()
        ctx.check()
        a = acc.cpu().numpy().astype(np.float64)[np.asarray(sample)]
        ref = np.asarray(a_ref, np.float64)
        return float(np.median(np.linalg.norm(a - ref, axis=1) / np.linalg.norm(ref, axis=1)))
    finally:
        ctx.set_tuning(chunk=old.chunk, blocks_per_cu=old.blocks_per_cu, lpt=old.lpt, tile=old.tile)


def autotune_learned(tree: Tree, eps: float, theta: float, ctx: Context, net, sample, a_ref,
                     ratios=NEAR_RATIOS, err_target: float = ERR_TARGET, grid=None, reps: int = 10, log=None):
    """The learned step on near cells tuned with an accuracy bound: for each
    near ratio the fastest group size and schedule (autotune with the
    correction in the timed step), then the step's median error at the sample
    with that schedule; the choice is choose_near_ratio's.  Returns (best
    dict with near_ratio, median_err and err_target, rows of every ratio)."""
    rows = []
    for r in ratios:
        best, _ = autotune(tree, eps, theta, ctx, grid=grid, reps=reps, log=log, corr_kind=CORR_MLP, net=net,
                           near_ratio=r)
        err = step_median_error(ctx, tree, eps, theta, best, net, r, sample, a_ref)
        rows.append(dict(best, near_ratio=r, median_err=err))
        if log:
            log(f"  near ratio {r}: {best['group_mode']} {best['g_max']}, {best['ms']:.3f} ms, median error {err:.3e}")
    return dict(choose_near_ratio(rows, err_target), err_target=err_target), rows


def load_cache(path: str = DEFAULT_CACHE) -> dict:
    if os.path.exists(path):
        with open(path) as f:
            return json.load(f)
    return {}


def save_cache(entry_key: str, best: dict, path: str = DEFAULT_CACHE):
    cache = load_cache(path)
    cache[entry_key] = best
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


DEFAULT_SCHEDULE = dict(group_mode="chunk", g_max=64, chunk=2048, blocks_per_cu=8, lpt=1, tile=256)


def cache_key(workload: str, mode: str = "plain", device: int = 0) -> str:
    """Cache key of a workload's schedule: the plain force, or the corrected
    step of mode "quad", "learned" (network on the near cells) or
    "learned-all" (network on every cell), each with its own best group size."""
    return f"{device_key(device)}:{workload}" + ("" if mode == "plain" else f"+{mode}")


def cached_schedule(workload: str, device: int = 0, path: str = DEFAULT_CACHE, mode: str = "plain"):
    """(schedule, source): the cached choice for this device, workload and
    mode; for a corrected mode without its own entry, the plain force's; else
    the defaults."""
    sched = dict(DEFAULT_SCHEDULE)
    cache = load_cache(path)
    cached = cache.get(cache_key(workload, mode, device))
    source = "autotune cache" + ("" if mode == "plain" else f" ({mode} step)")
    if not cached and mode != "plain":
        cached = cache.get(cache_key(workload, "plain", device))
        source = "autotune cache (plain force)"
    if not cached:
        return sched, "defaults"
    sched.update({k: cached[k] for k in sched})
    return sched, source


def cached_near_ratio(workload: str, device: int = 0, path: str = DEFAULT_CACHE, default: float = 0.4) -> float:
    """The near ratio of the cached learned step (near cells) of this device
    and workload, or `default`."""
    cached = load_cache(path).get(cache_key(workload, "learned", device)) or {}
    return float(cached.get("near_ratio", default))


def apply_schedule(ctx: Context, sched: dict):
    """Set the device half of a schedule on a context."""
    ctx.set_tuning(chunk=int(sched["chunk"]), blocks_per_cu=int(sched["blocks_per_cu"]), lpt=int(sched["lpt"]),
                   tile=int(sched["tile"]))

