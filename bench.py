"""Benchmark: Ginteractions/s and ms per full force evaluation on one MI355X.

Default workload: Plummer sphere, N = 2^20 equal masses (G = M = a = 1), seed 1,
softening 0.005, opening angle 0.5, groups of at most g_max particles.  The
host builds the tree and walks it once (timed separately, like the paper's
TREE / KERNEL / PCIe breakdown); the lists are uploaded once; a step is one
full force evaluation on the device (pack, schedule, force kernel, reduction)
replayed from a captured HIP graph with all inputs resident in HBM.

    python bench.py [--gpus 1] [--steps 20] [--warmup 3] [--workload plummer1m]

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Ginteractions/s and ms per full force eval at 1e-3 median force error, 1 GPU"
FLOPS_PER_INTERACTION = 20          # the paper's counting convention (Sec. 5)
PEAK_FP32_TFLOPS = 157.3            # MI355X FP32 vector peak (packed); 78.6 without packed FP32

WORKLOADS = {
    # name: (generator, kwargs, eps, theta, default g_max, description)
    "plummer16k": ("plummer", dict(n=16384, seed=0), 0.01, 0.5, 64,
                   "Plummer N=16384 seed=0 eps=0.01 theta=0.5"),
    "plummer1m": ("plummer", dict(n=1 << 20, seed=1), 0.005, 0.5, 64,
                  "Plummer N=1048576 seed=1 eps=0.005 theta=0.5"),
    "polytrope2m": ("polytrope_pair", dict(n_each=1 << 20, seed=2), 1e-4, 0.6, 64,
                    "two n=1.5 polytropes 2x1048576 seed=2 eps=1e-4 theta=0.6"),
    "cube16m": ("grf_cube", dict(ng=256, seed=4), 1e-3, 0.7, 256,
                "GRF cube 256^3 P(k)~k^-2 rms 0.3 seed=4 eps=1e-3 theta=0.7"),
}


def make_workload(name):
    import synth
    gen, kw, eps, theta, g_max, desc = WORKLOADS[name]
    out = getattr(synth, gen)(**kw)
    pos, m = out[0], out[1]
    return pos, m, eps, theta, g_max, desc


def cpu_baseline(pos32, mass32, lists, cm, eps, acc_gpu, pot_gpu, pos64_sorted, m64_sorted, sample_seed):
    """The FP64 oracle timed on this host (all targets of the workload), plus
    accuracy: GPU vs the oracle's list sums (parity) and the tree force vs the
    O(N^2) direct sum on a 4096-particle sample."""
    import oracle
    oracle.build()
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    t0 = time.perf_counter()
    a_ref, p_ref = oracle.list_force(pos32.astype(np.float64), mass32.astype(np.float64), lists.group_off,
                                     lists.list_off, lists.list_idx, cm[:, :3].astype(np.float64),
                                     cm[:, 3].astype(np.float64), float(np.float32(eps)))
    dt = time.perf_counter() - t0
    ea = oracle.rel_err(acc_gpu, a_ref)
    ep = oracle.rel_err(pot_gpu, p_ref)
    import synth
    sample = synth.sample_idx(len(mass32), 4096, seed=sample_seed)
    a_dir, p_dir = oracle.direct(pos64_sorted, m64_sorted, eps, tgt=sample)
    et = oracle.rel_err(acc_gpu[sample], a_dir)
    ept = oracle.rel_err(pot_gpu[sample], p_dir)
    base = {"value": lists.interactions / dt / 1e9, "unit": "Ginteractions/s", "cores": threads, "kind": "oracle",
            "sample": f"FP64 list sums over all {len(mass32)} targets ({lists.interactions} interactions), "
                      f"{dt:.2f} s"}
    acc = {"parity_acc_median": float(np.median(ea)), "parity_acc_max": float(ea.max()),
           "parity_pot_median": float(np.median(ep)), "parity_pot_max": float(ep.max()),
           "tree_acc_median_vs_direct": float(np.median(et)), "tree_acc_p99_vs_direct": float(np.quantile(et, 0.99)),
           "tree_pot_median_vs_direct": float(np.median(ept)), "direct_sample": 4096}
    return base, acc


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="plummer1m", choices=sorted(WORKLOADS))
    ap.add_argument("--g-max", type=int, default=0)
    ap.add_argument("--group-mode", default="chunk", choices=["chunk", "cell"])
    ap.add_argument("--chunk", type=int, default=1024)
    ap.add_argument("--blocks-per-cu", type=int, default=8)
    ap.add_argument("--lpt", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--quiet", action="store_true")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path (run with --gpus 1)",
              file=sys.stderr)
        sys.exit(2)

    def log(*a):
        if not args.quiet:
            print(*a, file=sys.stderr, flush=True)

    import torch
    import paper_1206_1199_amd as otoo

    pos, m, eps, theta, g_max, desc = make_workload(args.workload)
    if args.g_max:
        g_max = args.g_max
    mode = otoo.GROUP_CHUNK if args.group_mode == "chunk" else otoo.GROUP_CELL
    log(f"workload {desc}: n={len(m)}")

    t0 = time.perf_counter()
    tree = otoo.Tree(pos, m, n_crit=16)
    t1 = time.perf_counter()
    lists = tree.walk(theta=theta, g_max=g_max, group_mode=mode)
    t2 = time.perf_counter()
    perm, pos32, mass32, cm = tree.export(4)
    log(f"tree {1e3 * (t1 - t0):.0f} ms, walk {1e3 * (t2 - t1):.0f} ms: groups {lists.n_groups}, "
        f"entries {lists.n_entries}, interactions {lists.interactions}")

    torch.cuda.synchronize()
    t3 = time.perf_counter()
    d = otoo.DeviceLists.from_host(pos32, mass32, lists, cm, "cuda:0")
    torch.cuda.synchronize()
    t4 = time.perf_counter()

    ctx = otoo.Context(0)
    ctx.set_tuning(chunk=args.chunk, blocks_per_cu=args.blocks_per_cu, lpt=args.lpt)
    out = ctx.outputs(d.n)

    # kernel duration, measured with HIP events on the stream the kernel runs on
    ctx.enable_timing(True)
    kms = []
    for _ in range(max(3, args.warmup)):
        ctx.force(d, eps, out=out)
        kms.append(ctx.last_timing())
    kms = []
    for _ in range(max(5, min(args.steps, 20))):
        ctx.force(d, eps, out=out)
        kms.append(ctx.last_timing())
    ctx.enable_timing(False)
    ctx.check()
    k_ms = float(np.mean([k for k, _ in kms]))

    # the timed steps: graph replays
    ctx.graph_capture(d, eps, out)
    for _ in range(args.warmup):
        ctx.graph_launch()
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    w0 = time.perf_counter()
    e0.record(stream)
    for _ in range(args.steps):
        ctx.graph_launch()
    e1.record(stream)
    torch.cuda.synchronize()
    w1 = time.perf_counter()
    ms = e0.elapsed_time(e1) / args.steps
    ctx.check()
    log(f"force eval {ms:.3f} ms/step (wall {1e3 * (w1 - w0) / args.steps:.3f}), force kernel {k_ms:.3f} ms")

    acc = out[0].cpu().numpy().astype(np.float64)
    pot = out[1].cpu().numpy()
    inter = lists.interactions
    achieved = FLOPS_PER_INTERACTION * inter / (k_ms * 1e-3) / 1e12
    res = {
        "metric": METRIC,
        "value": inter / (ms * 1e-3) / 1e9,
        "unit": "Ginteractions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": desc, "n": int(len(m)), "g_max": g_max, "group_mode": args.group_mode,
                   "groups": lists.n_groups, "list_entries": lists.n_entries, "interactions": inter,
                   "n_cells": tree.n_cells, "chunk": args.chunk, "blocks_per_cu": args.blocks_per_cu,
                   "lpt": args.lpt},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP32_TFLOPS, "traffic": None,
                     "kernel": "k_force", "kernel_ms": k_ms,
                     "flops_per_interaction": FLOPS_PER_INTERACTION},
        "host": {"tree_build_ms": 1e3 * (t1 - t0), "walk_ms": 1e3 * (t2 - t1), "h2d_ms": 1e3 * (t4 - t3)},
    }
    if not args.no_cpu_baseline:
        pos_sorted = pos[perm]
        m_sorted = m[perm]
        sample_seed = {"plummer1m": 101, "polytrope2m": 102, "cube16m": 104}.get(args.workload, 100)
        base, accy = cpu_baseline(pos32, mass32, lists, cm, eps, acc, pot, pos_sorted, m_sorted, sample_seed)
        res["cpu_baseline"] = base
        res["accuracy"] = accy
        log(f"accuracy {accy}")
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
