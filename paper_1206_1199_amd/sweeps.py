"""Cost/accuracy sweeps of the walk settings over the paper's test
distributions: the absolute MAC (Sec. 2.2, Eq. 1, with m_limit) as a
function of its accuracy parameter Delta on the uniform sphere and the
Plummer model of Sec. 4.3-4.4, and the opening angle of the BH MAC.

For every setting: host walk time, interactions, the device force time (the
mean of captured-graph replays with inputs in HBM) and the relative
acceleration error against FP64 direct sums at a 4096-particle sample (mean,
the paper's "average error", and median).  The fitted log-log slopes of time
and error against Delta over the small-Delta end are printed at the end; the
paper's models are Delta^-3/4 for the cost and Delta^1/4 for the error.

    python -m paper_1206_1199_amd.sweeps delta [--dist uniform|plummer] [--n N] [--eps E]
    python -m paper_1206_1199_amd.sweeps theta [--dist ...]
    python -m paper_1206_1199_amd.sweeps sph [--dist polytrope|uniform|plummer] [--n N] [--k K]
    python -m paper_1206_1199_amd.sweeps corr [--dist plummer|cube] [--n N] [--values THETA] [--gates G,...]
                                              [--group-mode chunk|cell] [--net-kernels K,...]

The sph sweep times the SPH neighbour walk and the gather sums (density,
q = m) with neighbour radii from the K-th nearest neighbour, for each g_max.
The corr sweep times the cell-correction passes on the lists of one opening
angle: the textbook quadrupole and the network at each gate and with each
network kernel (the network's initial parameters: the gate depends on the
features only, so the cost is that of a trained network).  The cube
distribution is the GRF cube of (N^(1/3))^3 particles.

One JSON object per setting on stdout; a summary object last.
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np

from . import GROUP_CELL, GROUP_CHUNK, MAC_ABSOLUTE, MAC_BH, Context, DeviceLists, Tree

DELTAS = (1.0, 0.3, 0.1, 0.03, 0.01, 0.003, 0.001, 3e-4)
THETAS = (0.3, 0.4, 0.5, 0.6, 0.7, 0.8, 0.9)


def _schedule(ctx: Context, g_max: int):
    # whole lists per item for small groups, split lists and longest-first for large ones
    if g_max <= 32:
        ctx.set_tuning(chunk=1 << 24, blocks_per_cu=8, lpt=0, tile=512)
    else:
        ctx.set_tuning(chunk=2048, blocks_per_cu=8, lpt=1, tile=256)


def _time_force(ctx: Context, d: DeviceLists, eps: float, reps: int):
    import torch
    out = ctx.outputs(d.n)
    ctx.force(d, eps, out=out)
    ctx.graph_capture(d, eps, out)
    for _ in range(2):
        ctx.graph_launch()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        ctx.graph_launch()
    e1.record()
    torch.cuda.synchronize()
    ctx.check()
    return e0.elapsed_time(e1) / reps, out


def _slope(xs, ys):
    lx, ly = np.log(np.asarray(xs, float)), np.log(np.asarray(ys, float))
    return float(np.polyfit(lx, ly, 1)[0])


def run(kind: str, dist: str, n: int, eps: float, g_list, values, m_limit: float, reps: int, seed: int,
        emit=print):
    import torch
    import synth
    if dist == "uniform":
        pos, m = synth.uniform_sphere(n, seed=seed)
    else:
        pos, m = synth.plummer(n, seed=seed)
    t0 = time.perf_counter()
    tree = Tree(pos, m, n_crit=16)
    t_build = time.perf_counter() - t0
    perm, pos32, mass32, cm = tree.export(4)
    ctx = Context(0)
    sample = synth.sample_idx(n, 4096, seed=seed + 100)
    dev = "cuda:0"
    pos_t = torch.from_numpy(pos32).to(dev)
    mass_t = torch.from_numpy(mass32).to(dev)
    a_dir, _ = ctx.direct(pos_t, mass_t, torch.from_numpy(sample.astype(np.int32)).to(dev), eps)
    a_dir = a_dir.cpu().numpy()
    ctx.check()
    rows = []
    for g_max in g_list:
        _schedule(ctx, g_max)
        for v in values:
            t0 = time.perf_counter()
            if kind == "delta":
                lists = tree.walk(g_max=g_max, group_mode=GROUP_CHUNK, mac=MAC_ABSOLUTE, delta=v, m_limit=m_limit)
            else:
                lists = tree.walk(theta=v, g_max=g_max, group_mode=GROUP_CHUNK, mac=MAC_BH)
            t_walk = time.perf_counter() - t0
            d = DeviceLists.from_host(pos32, mass32, lists, cm, dev)
            ms, out = _time_force(ctx, d, eps, reps)
            acc = out[0][torch.from_numpy(sample).to(dev)].double().cpu().numpy()
            err = np.linalg.norm(acc - a_dir, axis=1) / np.linalg.norm(a_dir, axis=1)
            row = {kind: v, "g_max": g_max, "walk_s": t_walk, "force_ms": ms, "interactions": lists.interactions,
                   "list_entries": lists.n_entries, "groups": lists.n_groups,
                   "gint_per_s": lists.interactions / (ms * 1e-3) / 1e9, "mean_err": float(err.mean()),
                   "median_err": float(np.median(err)), "p99_err": float(np.quantile(err, 0.99))}
            rows.append(row)
            emit(json.dumps(row))
            sys.stdout.flush()
            del d, out
            torch.cuda.empty_cache()
    summary = {"sweep": kind, "dist": dist, "n": n, "eps": eps, "m_limit": m_limit if kind == "delta" else None,
               "tree_build_s": t_build, "n_cells": tree.n_cells}
    if kind == "delta":
        for g_max in g_list:
            small = [r for r in rows if r["g_max"] == g_max and r["delta"] <= 0.01]
            if len(small) >= 2:
                summary[f"g{g_max}_time_slope"] = _slope([r["delta"] for r in small], [r["force_ms"] for r in small])
                summary[f"g{g_max}_err_slope"] = _slope([r["delta"] for r in small], [r["mean_err"] for r in small])
    emit(json.dumps(summary))
    return rows, summary


def run_sph(dist: str, n: int, g_list, k: int, reps: int, seed: int, emit=print):
    import torch
    import synth
    if dist == "polytrope":
        pos, m, _, _ = synth.polytrope_pair(n // 2, seed=seed)
    elif dist == "uniform":
        pos, m = synth.uniform_sphere(n, seed=seed)
    else:
        pos, m = synth.plummer(n, seed=seed)
    h = synth.knn_radius(pos, k)
    tree = Tree(pos, m, n_crit=16)
    perm, pos32, mass32, cm = tree.export(4)
    ctx = Context(0)
    dev = "cuda:0"
    h_t = torch.from_numpy(h[perm].astype(np.float32)).to(dev)
    q_t = torch.from_numpy(mass32).to(dev)
    rows = []
    for g_max in g_list:
        t0 = time.perf_counter()
        lists = tree.walk_sph(h, g_max=g_max)
        t_walk = time.perf_counter() - t0
        d = DeviceLists.from_host(pos32, mass32, lists, cm, dev)
        out = ctx.sph_sum(d, h_t, q_t)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            ctx.sph_sum(d, h_t, q_t, out=out)
        e1.record()
        torch.cuda.synchronize()
        ctx.check()
        ms = e0.elapsed_time(e1) / reps
        row = {"sph": dist, "n": len(m), "k": k, "g_max": g_max, "walk_s": t_walk, "sum_ms": ms,
               "pairs": lists.interactions, "list_entries": lists.n_entries,
               "gpairs_per_s": lists.interactions / (ms * 1e-3) / 1e9}
        rows.append(row)
        emit(json.dumps(row))
        sys.stdout.flush()
        del d
        torch.cuda.empty_cache()
    return rows


def run_corr(dist: str, n: int, g_list, theta: float, gates, eps: float, reps: int, seed: int, emit=print,
             group_mode: int = GROUP_CHUNK, net_kernels=(0,)):
    import torch
    import synth
    from . import CORR_MLP, CORR_QUAD, learned
    if dist == "plummer":
        pos, m = synth.plummer(n, seed=seed)
    elif dist == "cube":
        pos, m = synth.grf_cube(int(round(n ** (1.0 / 3.0))), seed=seed)
    else:
        pos, m = synth.uniform_sphere(n, seed=seed)
    tree = Tree(pos, m, n_crit=16)
    _, pos32, mass32, cm = tree.export(12)
    ctx = Context(0)
    net = learned.Network(ctx)
    net.set_params(learned.init_params(0))
    rows = []

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        ctx.check()
        return e0.elapsed_time(e1) / reps

    old = ctx.tuning()
    for g_max in g_list:
        d = DeviceLists.from_host(pos32, mass32, tree.walk(theta=theta, g_max=g_max, group_mode=group_mode), cm,
                                  "cuda:0")
        out = ctx.correction(d, CORR_QUAD, eps)
        row = {"corr": dist, "n": len(m), "theta": theta, "g_max": g_max,
               "group_mode": "chunk" if group_mode == GROUP_CHUNK else "cell", "pairs": d.n_pairs,
               "quad_ms": timed(lambda: ctx.correction(d, CORR_QUAD, eps, out=out))}
        for kernel in net_kernels:
            ctx.set_tuning(net_kernel=kernel)
            for gate in gates:
                net.set_gate(gate)
                key = f"net_ms_gate_{gate:g}" if len(net_kernels) == 1 else f"net{kernel}_ms_gate_{gate:g}"
                row[key] = timed(lambda: ctx.correction(d, CORR_MLP, eps, net=net, out=out))
        ctx.set_tuning(net_kernel=old.net_kernel)
        rows.append(row)
        emit(json.dumps(row))
        sys.stdout.flush()
    return rows


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("kind", choices=["delta", "theta", "sph", "corr"])
    ap.add_argument("--dist", choices=["uniform", "plummer", "polytrope", "cube"], default="uniform")
    ap.add_argument("--k", type=int, default=50, help="sph: neighbours inside h")
    ap.add_argument("--n", type=int, default=8000 * 1024)
    ap.add_argument("--eps", type=float, default=1e-3)
    ap.add_argument("--g-max", default="32,64")
    ap.add_argument("--values", default="", help="comma-separated Delta (or theta) values")
    ap.add_argument("--m-limit", type=float, default=0.05)
    ap.add_argument("--reps", type=int, default=5)
    ap.add_argument("--seed", type=int, default=5)
    ap.add_argument("--gates", default="0.4,0", help="corr: network gates (l/|d| thresholds)")
    ap.add_argument("--group-mode", choices=["chunk", "cell"], default="chunk", help="corr: how groups are formed")
    ap.add_argument("--net-kernels", default="", help="corr: network kernels to time (default: the context's)")
    a = ap.parse_args(argv)
    if a.kind == "corr":
        theta = float(a.values) if a.values else 0.9
        kernels = [int(k) for k in a.net_kernels.split(",")] if a.net_kernels else [Context(0).tuning().net_kernel]
        run_corr(a.dist, a.n, [int(g) for g in a.g_max.split(",")], theta, [float(x) for x in a.gates.split(",")],
                 a.eps, a.reps, a.seed, group_mode=GROUP_CHUNK if a.group_mode == "chunk" else GROUP_CELL,
                 net_kernels=kernels)
        return
    if a.kind == "sph":
        run_sph(a.dist, a.n, [int(g) for g in a.g_max.split(",")], a.k, a.reps, a.seed)
        return
    values = [float(x) for x in a.values.split(",")] if a.values else (DELTAS if a.kind == "delta" else THETAS)
    run(a.kind, a.dist, a.n, a.eps, [int(g) for g in a.g_max.split(",")], values, a.m_limit, a.reps, a.seed)


if __name__ == "__main__":
    main()
