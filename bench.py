"""Benchmark: Ginteractions/s and ms per full force evaluation on one MI355X.

Default workload: the isolated GRF cube of 256^3 = 2^24 particles (P(k) ~ k^-2,
rms 0.3, seed 4), softening 1e-3, opening angle 0.7, with the learned cell
correction and FP32 + Kahan sums: the largest single-GPU configuration.  The
host builds the tree and walks it once (timed separately, like the paper's
TREE / KERNEL / PCIe breakdown); the lists are uploaded once; the network is
trained here on the GPU from the method's own walks; a step is one full force
evaluation on the device -- the learned correction pass (features, gated
network, per-group local expansion) and the force (pack, schedule, force
kernel, reduction) -- captured in one graph and replayed with every input
resident in HBM.

    python bench.py [--gpus 1] [--steps 20] [--warmup 10] [--workload cube16m]
                    [--mode plain|quad|learned] [--autotune] [--no-learned]
                    [--no-cpu-baseline] [--no-plummer]

Other workloads (plummer1m, polytrope2m, plummer16k) default to the plain
monopole force.  The line also carries the Plummer 2^20 plain headline
(skip with --no-plummer) and the learned-correction comparison on a held-out
Plummer sphere at equal 1e-3 median error (skip with --no-learned).

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import contextlib
import json
import os
import sys
import time
import types

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Ginteractions/s and ms per full force eval at 1e-3 median force error, 1 GPU"
FLOPS_PER_INTERACTION = 20          # the paper's counting convention (Sec. 5)
PEAK_FP32_TFLOPS = 157.3            # MI355X FP32 vector peak (packed)
PEAK_FP32_NONPACKED_TFLOPS = 78.6   # 256 CU x 64 lanes x 2 flops (FMA) x 2.4 GHz, one FP32 op per lane per clock

WORKLOADS = {
    # name: (generator, kwargs, eps, theta, description)
    "plummer16k": ("plummer", dict(n=16384, seed=0), 0.01, 0.5, "Plummer N=16384 seed=0 eps=0.01 theta=0.5"),
    "plummer1m": ("plummer", dict(n=1 << 20, seed=1), 0.005, 0.5, "Plummer N=1048576 seed=1 eps=0.005 theta=0.5"),
    "polytrope2m": ("polytrope_pair", dict(n_each=1 << 20, seed=2), 1e-4, 0.6,
                    "two n=1.5 polytropes 2x1048576 seed=2 eps=1e-4 theta=0.6"),
    "cube16m": ("grf_cube", dict(ng=256, seed=4), 1e-3, 0.7,
                "GRF cube 256^3 P(k)~k^-2 rms 0.3 seed=4 eps=1e-3 theta=0.7"),
}
SAMPLE_SEED = {"plummer16k": 100, "plummer1m": 101, "polytrope2m": 102, "cube16m": 104}
# group sizes the workload allows the autotuner (the 2^20 Plummer sphere is
# quoted with groups of 64-256 particles, the 16k sphere with groups <= 64)
# Group choices the autotuner may take per workload.  The 2^20 Plummer
# workload fixes groups of 64-256 particles: chunk groups of exactly 64, 128
# or 256 (a cell group of g_max holds anywhere from 1 to g_max particles).
GROUPS = {
    "plummer16k": [(0, 64), (1, 64)],
    "plummer1m": [(0, 64), (0, 128), (0, 256)],
}


@contextlib.contextmanager
def marker(name):
    """A roctx range around a host phase (torch's NVTX calls are roctx on
    ROCm), shown by a rocprofv3 marker trace; a no-op where markers are
    unavailable."""
    try:
        import torch
        torch.cuda.nvtx.range_push(name)
        pushed = True
    except Exception:
        pushed = False
    try:
        yield
    finally:
        if pushed:
            torch.cuda.nvtx.range_pop()


def measured_traffic(workload, mode, desc, sched):
    """HBM bytes per force-kernel launch from the committed rocprofv3 counter
    summary of this workload and mode (profiles/k_force_<workload>[_<mode>].md),
    when it was taken on this workload and schedule with the current kernel
    source; otherwise None."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"k_force_{workload}" + ("" if mode == "plain" else f"_{mode}") + ".md")
    if not os.path.exists(path):
        return None
    fields = {}
    for line in open(path):
        if ":" in line and line.split(":", 1)[0] in ("traffic_bytes_per_launch", "source_sha256", "workload",
                                                     "schedule"):
            k, v = line.split(":", 1)
            fields[k] = v.strip()
    h = hashlib.sha256()
    for f in ("paper_1206_1199_amd/csrc/otoo_force.hip", "paper_1206_1199_amd/csrc/otoo_internal.h"):
        h.update(open(os.path.join(ROOT, f), "rb").read())
    if (fields.get("source_sha256") == h.hexdigest()[:16] and fields.get("workload") == desc
            and fields.get("schedule") == json.dumps(sched, sort_keys=True)):
        return float(fields["traffic_bytes_per_launch"])
    return None


def particle_classes(name, out):
    """Boolean masks over the input order for the workload's particle classes
    (the polytrope pair: star A, star B, and cores r < R/4 vs envelopes)."""
    if name != "polytrope2m":
        return {}
    pos, _, star, centres = out
    radius = np.where(star == 0, 0.02, 0.012)
    r = np.linalg.norm(pos - centres[star], axis=1)
    core = r < radius / 4
    return {"A": star == 0, "B": star == 1, "core": core, "envelope": ~core}


def make_workload(name):
    import synth
    gen, kw, eps, theta, desc = WORKLOADS[name]
    out = getattr(synth, gen)(**kw)
    return out[0], out[1], eps, theta, desc, particle_classes(name, out)


# ------------------------------------------------------------------ CPU baseline leg (the oracle)


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _omp_threads(k):
    """Set the OpenMP thread count of the oracle's runtime (libgomp)."""
    import ctypes
    ctypes.CDLL("libgomp.so.1").omp_set_num_threads(int(k))


def cpu_baseline(pos32, mass32, lists, cm, eps, sample=None):
    """The FP64 oracle timed on this host: list sums for every target on all
    cores (same FP32 inputs and lists as the device), the same sums for every
    16th group on one core, and the O(N^2) direct sum at the accuracy sample.

    Returns (baseline dict, list-sum references (acc, pot), direct sums at the
    sample or None)."""
    import oracle
    oracle.build()
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    p64, m64 = pos32.astype(np.float64), mass32.astype(np.float64)
    com, cmass, e = cm[:, :3].astype(np.float64), cm[:, 3].astype(np.float64), float(np.float32(eps))
    t0 = time.perf_counter()
    ref = oracle.list_force(p64, m64, lists.group_off, lists.list_off, lists.list_idx, com, cmass, e)
    dt = time.perf_counter() - t0
    base = {"value": lists.interactions / dt / 1e9, "unit": "Ginteractions/s", "cores": threads, "kind": "oracle",
            "sample": f"FP64 list sums over all {len(mass32)} targets of the workload "
                      f"({lists.interactions} interactions) in {dt:.2f} s",
            "cpu": _cpu_model(), "nproc": os.cpu_count()}
    # one core, every 16th group
    go, lo = np.asarray(lists.group_off, np.int64), np.asarray(lists.list_off, np.int64)
    groups = np.arange(0, len(go) - 1, 16)
    tgt = np.concatenate([np.arange(go[g], go[g + 1]) for g in groups])
    inter1 = int(((go[groups + 1] - go[groups]) * (lo[groups + 1] - lo[groups])).sum())
    _omp_threads(1)
    try:
        t0 = time.perf_counter()
        oracle.list_force(p64, m64, lists.group_off, lists.list_off, lists.list_idx, com, cmass, e, tgt=tgt)
        dt1 = time.perf_counter() - t0
    finally:
        _omp_threads(threads)
    base["one_core"] = {"value": inter1 / dt1 / 1e9, "unit": "Ginteractions/s", "cores": 1,
                        "sample": f"every 16th group ({len(groups)} groups, {len(tgt)} targets, {inter1} "
                                  f"interactions) in {dt1:.2f} s"}
    direct = None
    if sample is not None:
        t0 = time.perf_counter()
        direct = oracle.direct(p64, m64, e, tgt=np.asarray(sample, np.int64))
        dtd = time.perf_counter() - t0
        pairs = len(sample) * len(mass32)
        base["direct"] = {"value": pairs / dtd / 1e9, "unit": "Gpairs/s", "cores": threads,
                          "sample": f"O(N^2) FP64 sums at {len(sample)} targets ({pairs} pairs) in {dtd:.2f} s"}
    return base, ref, direct


def direct_reference(ctx, d, sample, eps):
    """FP64 direct sums on the device at the sample (indices in device order)."""
    import torch
    tgt = torch.from_numpy(np.asarray(sample, np.int32)).to(d.pos.device)
    a, p = ctx.direct(d.pos, d.mass, tgt, eps)
    torch.cuda.synchronize()
    ctx.check()
    return a.cpu().numpy(), p.cpu().numpy()


def rel_err(a, ref):
    a = np.asarray(a, np.float64)
    ref = np.asarray(ref, np.float64)
    if a.ndim == 2:
        return np.linalg.norm(a - ref, axis=1) / np.linalg.norm(ref, axis=1)
    return np.abs(a - ref) / np.abs(ref)


# ------------------------------------------------------------------ learned comparison


def train_network(ctx, log, train_steps, gate=0.4, near=True):
    """Train the correction network on the GPU on samples of seeded walks of
    Plummer spheres and GRF cubes; returns (net, summary).  near: the samples are the near pairs
    (l/|COM - c_g| >= gate), which the walks list first and which alone get
    the correction, and the network runs on every pair it is given (device
    gate 0); else the layers are gated to pairs with BF16 l/n >= gate and the
    other pairs keep the textbook quadrupole."""
    import torch
    from paper_1206_1199_amd import learned
    eps = 0.005
    net = learned.Network(ctx)
    net.set_params(learned.init_params(0))
    net.set_gate(0.0 if near else gate)
    keep = 3 if (gate > 0 and not near) else 1   # draws per kept sample: the gate passes about a third of the pairs
    rng = np.random.Generator(np.random.PCG64(12345))
    cfgs = [learned.SampleConfig("plummer", 16384, 1000 + k, 0.01, float(rng.uniform(0.5, 1.0)), 64, 40000 * keep)
            for k in range(20)]
    cfgs += [learned.SampleConfig("plummer", 1 << 20, 1020 + k, eps, float(rng.uniform(0.5, 1.0)),
                                  int(rng.choice([32, 64, 128])), 240000 * keep) for k in range(5)]
    # GRF cubes of 64^3 and 128^3 particles (seeds 2000+, never the benchmark cube's), softening a
    # quarter of the lattice spacing
    cfgs += [learned.SampleConfig("grf_cube", ng ** 3, 2000 + k, 0.25 / ng, float(rng.uniform(0.6, 1.0)),
                                  int(rng.choice([32, 64, 128])), 133000 * keep)
             for k, ng in enumerate((64, 128, 64, 128, 64, 128, 64, 128))]
    t0 = time.perf_counter()
    X, aux, eps_all = learned.make_training_set(ctx, net, cfgs, seed=1, gate=gate, near=near)
    Xv, auxv, epsv = learned.make_training_set(
        ctx, net, [learned.SampleConfig("plummer", 1 << 20, 1100, eps, 0.9, 64, 100000 * keep)], seed=2, gate=gate,
        near=near)
    t_data = time.perf_counter() - t0
    base_val = learned.zero_correction_loss(auxv)
    net.set_params(np.zeros(learned.N_PARAMS, np.float32))
    quad_val = learned.evaluate_loss(net, Xv, auxv, epsv)
    net.set_params(learned.init_params(0))
    t0 = time.perf_counter()
    learned.fit(net, X, aux, eps_all, steps=train_steps, batch=32768, lr=2e-3, seed=0, X_val=Xv, aux_val=auxv,
                eps_val=epsv, log=log, log_every=max(1, train_steps // 5))
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    val = learned.evaluate_loss(net, Xv, auxv, epsv)
    log(f"learned: {X.shape[0]} samples (gate {gate}, {'near pairs' if near else 'all pairs'}) in {t_data:.1f} s, "
        f"{train_steps} steps in {t_train:.1f} s, validation loss {val:.3e} (plain monopole {base_val:.3e}, textbook "
        f"quadrupole {quad_val:.3e})")
    return net, {"gate": gate, "pairs": "near" if near else "all", "samples": int(X.shape[0]), "steps": train_steps,
                 "data_s": t_data,
                 "train_s": t_train, "val_loss": val, "val_loss_plain_monopole": base_val,
                 "val_loss_textbook_quadrupole": quad_val}


def workload_learned(ctx, net, training, log, tree, eps, theta, scheds, sample, a_dir, reps, near_ratios=(0.0,)):
    """Plain, textbook-quadrupole and learned force on the benchmark workload
    itself, over opening angles around its own (plain at and below it, the
    corrections at and above it), each mode with its own cached schedule
    (``scheds[mode]``: the plain force's, or the corrected step's, whose best
    group size differs).  Each step (correction + force) is captured in one
    graph and replayed; errors are against the direct sums of the sample.
    near_ratios (> 0): the learned step corrects only the near cells (walks
    that list them first), at each of these ratios."""
    import torch
    import paper_1206_1199_amd as otoo
    from paper_1206_1199_amd import learned
    steps = lambda lo, hi: [round(theta + 0.05 * k, 2) for k in range(lo, hi + 1)]
    thetas = {"plain": steps(-2, 0), "quad": steps(-2, 1), "learned": steps(0, 6)}
    old = ctx.tuning()
    rows = []
    try:
        for mode in ("plain", "quad", "learned"):
            sc = scheds[mode]
            ctx.set_tuning(chunk=sc["chunk"], blocks_per_cu=sc["blocks_per_cu"], lpt=sc["lpt"], tile=sc["tile"])
            mode_id = otoo.GROUP_CHUNK if sc["group_mode"] == "chunk" else otoo.GROUP_CELL
            for th, near_ratio in [(th, r) for th in thetas[mode] for r in (near_ratios if mode == "learned" else (0.0,))]:
                lists = tree.walk(theta=th, g_max=sc["g_max"], group_mode=mode_id, near_ratio=near_ratio)
                d, _, _ = learned.device_tree_arrays(tree, lists)
                out = ctx.outputs(d.n)
                gc = torch.empty((d.n_groups, otoo.CORR_STRIDE), dtype=torch.float32, device="cuda:0")
                g = ctx.capture(make_step(ctx, d, eps, mode, net, out, gc))
                g.replay()
                torch.cuda.synchronize()
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record()
                for _ in range(reps):
                    g.replay()
                e1.record()
                torch.cuda.synchronize()
                ctx.check()
                err = rel_err(out[0].cpu().numpy()[sample], a_dir)
                rows.append(dict(mode=mode, theta=th, group_mode=sc["group_mode"], g_max=sc["g_max"],
                                 near_ratio=near_ratio, ms=e0.elapsed_time(e1) / reps,
                                 interactions=lists.interactions, pairs=d.n_pairs,
                                 median_err=float(np.median(err)), p99_err=float(np.quantile(err, 0.99))))
                log(f"  {mode:8s} theta {th:.2f} {sc['group_mode']} {sc['g_max']}"
                    + (f" ratio {near_ratio:.2f}" if near_ratio > 0 else "") + " (graph replay): "
                    f"{rows[-1]['ms']:.3f} ms, median err {rows[-1]['median_err']:.2e}")
                del g, d, out, gc
                torch.cuda.empty_cache()
    finally:
        ctx.set_tuning(chunk=old.chunk, blocks_per_cu=old.blocks_per_cu, lpt=old.lpt, tile=old.tile)
    ok = lambda mode: [r for r in rows if r["mode"] == mode and r["median_err"] <= 1e-3]
    best = {mode: (min(ok(mode), key=lambda r: r["ms"]) if ok(mode) else None) for mode in ("plain", "quad", "learned")}
    res = {"rows": rows, "best_at_1e-3": best}
    if best["learned"] and best["plain"]:
        res["learned_speedup_vs_best_plain"] = best["plain"]["ms"] / best["learned"]["ms"]
    return res


def learned_comparison(ctx, net, training, log, timing_reps):
    """Compare, on a held-out Plummer sphere (N = 2^20, seed 3, eps 0.005),
    plain theta = 0.5, plain at the largest theta with median error <= 1e-3,
    the textbook quadrupole and the learned correction, all timed per force
    evaluation with the best of a few schedules per setting.  A network
    trained on near pairs corrects the near cells of walks that list them
    first, at near ratio = its training gate and at 0.6."""
    import torch
    import synth
    import paper_1206_1199_amd as otoo
    from paper_1206_1199_amd import learned
    eps = 0.005
    gate = training["gate"]
    near_ratio = gate if training.get("pairs") == "near" else 0.0
    pos, m = synth.plummer(1 << 20, seed=3)
    tree = otoo.Tree(pos, m, n_crit=16)
    perm, pos32, mass32, cm = tree.export(12)
    sample = synth.sample_idx(len(m), 4096, seed=103)
    a_dir, _ = direct_reference(ctx, otoo.DeviceLists.from_host(pos32, mass32, tree.walk(theta=0.5), cm, "cuda:0"),
                                sample, eps)
    schedules = [dict(chunk=1 << 24, blocks_per_cu=8, lpt=0, tile=512), dict(chunk=2048, blocks_per_cu=8, lpt=1, tile=256),
                 dict(chunk=4096, blocks_per_cu=8, lpt=1, tile=512), dict(chunk=4096, blocks_per_cu=6, lpt=1, tile=256)]

    def timed(step):
        for _ in range(3):
            step()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(timing_reps):
            step()
        e1.record()
        torch.cuda.synchronize()
        ctx.check()
        return e0.elapsed_time(e1) / timing_reps

    def run(theta, modes, g_max, near_ratio=0.0):
        lists = tree.walk(theta=theta, g_max=g_max, near_ratio=near_ratio)
        d, _, _ = learned.device_tree_arrays(tree, lists)
        out = ctx.outputs(d.n)
        gc = torch.empty((d.n_groups, otoo.CORR_STRIDE), dtype=torch.float32, device="cuda:0")
        # the force schedule: the fastest candidate for this list set, shared by every mode
        best_s, best_ms = None, None
        for sc in schedules:
            ctx.set_tuning(**sc)
            ms = timed(lambda: ctx.force(d, eps, out=out))
            if best_ms is None or ms < best_ms:
                best_s, best_ms = sc, ms
        ctx.set_tuning(**best_s)
        rows = []
        for mode in modes:
            def step():
                if mode == "learned":
                    ctx.correction(d, otoo.CORR_MLP, eps, net=net, out=gc)
                    ctx.force(d, eps, out=out, gcorr=gc)
                elif mode == "quad":
                    ctx.correction(d, otoo.CORR_QUAD, eps, out=gc)
                    ctx.force(d, eps, out=out, gcorr=gc)
                else:
                    ctx.force(d, eps, out=out)
            ms = timed(step)
            err = rel_err(out[0].cpu().numpy()[sample], a_dir)
            rows.append(dict(mode=mode, theta=theta, g_max=g_max, near_ratio=near_ratio, ms=ms,
                             interactions=lists.interactions,
                             pairs=d.n_pairs, median_err=float(np.median(err)),
                             p99_err=float(np.quantile(err, 0.99)), schedule=best_s))
        return rows

    rows = []
    for th in (0.5, 0.6, 0.65, 0.7, 0.75, 0.8, 0.85, 0.9):
        rows += run(th, ("plain",), 32)
    for th in (0.5, 0.7, 0.75, 0.8):
        rows += run(th, ("plain",), 64)
    for g_max, ths in ((32, (0.8, 0.9)), (64, (0.8, 0.85, 0.9, 0.95, 1.0)), (128, (0.8, 0.85, 0.9, 0.95, 1.0))):
        for th in ths:
            rows += run(th, ("quad",), g_max)
            for ratio in ((near_ratio, 0.6) if near_ratio > 0 else (0.0,)):   # the training ratio, and 0.6
                rows += run(th, ("learned",), g_max, ratio)
    for r in rows:
        log(f"  {r['mode']:8s} g_max {r['g_max']:3d} theta {r['theta']:.2f}"
            + (f" ratio {r['near_ratio']:.2f}" if r["near_ratio"] > 0 else "")
            + f": {r['ms']:.3f} ms, median err {r['median_err']:.2e}, pairs {r['pairs']}")
    ok = lambda mode: [r for r in rows if r["mode"] == mode and r["median_err"] <= 1e-3]
    best = {mode: (min(ok(mode), key=lambda r: r["ms"]) if ok(mode) else None) for mode in ("plain", "quad", "learned")}
    plain05 = min((r for r in rows if r["mode"] == "plain" and r["theta"] == 0.5), key=lambda r: r["ms"])
    res = {"workload": "Plummer N=1048576 seed=3 eps=0.005 (held out), error vs direct sum on 4096 particles",
           "gate": gate, "learned_pairs": "near" if near_ratio > 0 else "all", "training": training, "plain_theta_0.5": plain05, "best_at_1e-3": best, "rows": rows}
    if best["learned"]:
        res["learned_speedup_vs_plain_theta_0.5"] = plain05["ms"] / best["learned"]["ms"]
        if best["plain"]:
            res["learned_speedup_vs_best_plain"] = best["plain"]["ms"] / best["learned"]["ms"]
    return res


# ------------------------------------------------------------------ the corrected step


HEADLINE_MODE = {"cube16m": "learned"}      # the cube is quoted with the learned correction


def make_step(ctx, d, eps, mode, net, out, gc):
    """One full force evaluation of the given mode (correction pass, if any,
    then the force), writing `out` (and the per-group expansion `gc`)."""
    import paper_1206_1199_amd as otoo
    if mode == "plain":
        return lambda: ctx.force(d, eps, out=out)
    kind = otoo.CORR_MLP if mode == "learned" else otoo.CORR_QUAD

    def step():
        ctx.correction(d, kind, eps, net=net, out=gc)
        ctx.force(d, eps, out=out, gcorr=gc)
    return step


def graph_kernel_ms(ctx, step, reps):
    """Mean duration of the force kernel inside replays of the step's graph:
    the library records HIP events around k_force on its stream, and with
    timing on they are captured into the graph as event nodes; each replay is
    synchronised and its event pair read.  None if the events cannot be
    captured."""
    import torch
    ctx.enable_timing(True)
    try:
        g = ctx.capture(step)
        g.replay()
        torch.cuda.synchronize()
        vals = []
        for _ in range(reps):
            g.replay()
            torch.cuda.synchronize()
            vals.append(ctx.last_timing()[0])
        ctx.check()
        return float(np.mean(vals))
    except Exception:
        return None
    finally:
        ctx.enable_timing(False)


def kernel_times(ctx, d, eps, mode, net, out, gc, reps):
    """Average durations of the force kernel (HIP events the library records
    around it on its stream) and of the correction pass (events on torch's
    current stream, which is the context's stream), from eager launches of
    the step's own calls."""
    import torch
    import paper_1206_1199_amd as otoo
    kind = otoo.CORR_MLP if mode == "learned" else otoo.CORR_QUAD
    kf, kc = [], []
    ctx.enable_timing(True)
    try:
        for r in range(reps + 2):
            if mode != "plain":
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record()
                ctx.correction(d, kind, eps, net=net, out=gc)
                e1.record()
                ctx.force(d, eps, out=out, gcorr=gc)
            else:
                ctx.force(d, eps, out=out)
            k, _ = ctx.last_timing()
            if r >= 2:
                kf.append(k)
                if mode != "plain":
                    kc.append(e0.elapsed_time(e1))
    finally:
        ctx.enable_timing(False)
    ctx.check()
    return float(np.mean(kf)), (float(np.mean(kc)) if kc else 0.0)


def time_graph(ctx, step, warmup, steps):
    """ms per step of `steps` replays of the step's graph (after `warmup`),
    bracketed by a device synchronisation on both sides, with HIP events on
    the replay stream."""
    import torch
    g = ctx.capture(step)
    for _ in range(warmup):
        g.replay()
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    with marker("timed force evaluations"):
        w0 = time.perf_counter()
        e0.record(stream)
        for _ in range(steps):
            g.replay()
        e1.record(stream)
        torch.cuda.synchronize()
        w1 = time.perf_counter()
    ctx.check()
    return e0.elapsed_time(e1) / steps, 1e3 * (w1 - w0) / steps


def cpu_baseline_corrected(pos32, mass32, lists, cm, eps, mode, params, gate, groups, tgt):
    """The FP64 oracle timed on this host for the corrected force of a sample
    of the workload's groups: the oracle's tensors of the sampled groups'
    (group, cell) pairs (textbook, or the FP64 network at the trained BF16
    weights) and its list sums with the cell tensors applied through the
    same local expansion, for every particle of those groups.  Returns
    (baseline dict, (acc, pot) at `tgt`)."""
    import oracle
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    from corr_parity import pair_tensors
    from learned_helpers import sub_lists
    oracle.build()
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    go = np.asarray(lists.group_off, np.int64)
    lo = np.asarray(lists.list_off, np.int64)
    all_t = np.concatenate([np.arange(go[g], go[g + 1]) for g in groups]).astype(np.int64)
    inter = int(((go[groups + 1] - go[groups]) * (lo[groups + 1] - lo[groups])).sum())
    p64, m64 = pos32.astype(np.float64), mass32.astype(np.float64)
    com, cmass, e = cm[:, :3].astype(np.float64), cm[:, 3].astype(np.float64), float(np.float32(eps))
    t0 = time.perf_counter()
    sub = sub_lists(lists, groups)
    Q, _ = pair_tensors("mlp" if mode == "learned" else "quad", lists, pos32, cm, eps, sub["pairs"], params, gate)
    acc, pot = oracle.list_force(p64, m64, sub["group_off"], sub["list_off"], sub["list_idx"], com, cmass, e,
                                 tgt=all_t, n_cellent=sub["n_cellent"], quad=Q, expanded=True)
    dt = time.perf_counter() - t0
    base = {"value": inter / dt / 1e9, "unit": "Ginteractions/s", "cores": threads, "kind": "oracle",
            "sample": f"FP64 oracle, {mode} correction: network/textbook tensors of {len(Q)} (group, cell) pairs "
                      f"and list sums with the expansion for all {len(all_t)} particles of {len(groups)} sampled "
                      f"groups ({inter} interactions) in {dt:.2f} s",
            "cpu": _cpu_model(), "nproc": os.cpu_count()}
    pos_of = {int(i): k for k, i in enumerate(all_t)}
    rows = np.array([pos_of[int(i)] for i in tgt], np.int64)
    return base, (acc[rows], pot[rows])


def plain_headline(ctx, log, steps, warmup, reps):
    """The plain monopole headline on the 2^20 Plummer sphere (theta 0.5, its
    cached schedule): ms per evaluation, interactions/s and the median error
    against direct sums at its 4096-particle sample."""
    import torch
    import paper_1206_1199_amd as otoo
    from paper_1206_1199_amd import autotune as at
    pos, m, eps, theta, desc, _ = make_workload("plummer1m")
    tree = otoo.Tree(pos, m, n_crit=16)
    sched, source = at.cached_schedule("plummer1m", 0)
    lists = tree.walk(theta=theta, g_max=sched["g_max"],
                      group_mode=otoo.GROUP_CHUNK if sched["group_mode"] == "chunk" else otoo.GROUP_CELL)
    _, pos32, mass32, cm = tree.export(4)
    d = otoo.DeviceLists.from_host(pos32, mass32, lists, cm, "cuda:0")
    old = ctx.tuning()
    ctx.set_tuning(chunk=sched["chunk"], blocks_per_cu=sched["blocks_per_cu"], lpt=sched["lpt"], tile=sched["tile"])
    try:
        out = ctx.outputs(d.n)
        step = make_step(ctx, d, eps, "plain", None, out, None)
        ms, _ = time_graph(ctx, step, warmup, steps)
        k_ms = graph_kernel_ms(ctx, step, reps)
        if k_ms is None:
            k_ms, _ = kernel_times(ctx, d, eps, "plain", None, out, None, reps)
    finally:
        ctx.set_tuning(chunk=old.chunk, blocks_per_cu=old.blocks_per_cu, lpt=old.lpt, tile=old.tile)
    sample = synth_sample(len(m), "plummer1m")
    a_dir, _ = direct_reference(ctx, d, sample, eps)
    err = rel_err(out[0].cpu().numpy()[sample], a_dir)
    res = {"workload": desc, "ms_per_step": ms, "value": lists.interactions / (ms * 1e-3) / 1e9,
           "unit": "Ginteractions/s", "interactions": lists.interactions, "schedule": sched,
           "k_force_ms": k_ms, "k_force_tflops": FLOPS_PER_INTERACTION * lists.interactions / (k_ms * 1e-3) / 1e12,
           "tree_acc_median_vs_direct": float(np.median(err))}
    log(f"plummer 2^20 plain: {ms:.3f} ms/step, {res['value']:.0f} Gint/s, median err {res['tree_acc_median_vs_direct']:.2e}")
    del d, out
    torch.cuda.empty_cache()
    return res


def workload_sample(workload, classes, perm, n):
    """The accuracy sample in device order: 4096 particles, or 2048 per star
    of the polytrope pair."""
    import synth
    seed = SAMPLE_SEED.get(workload, 100)
    if "A" in classes:
        ia, ib = np.flatnonzero(classes["A"][perm]), np.flatnonzero(classes["B"][perm])
        return np.concatenate([ia[synth.sample_idx(len(ia), 2048, seed)], ib[synth.sample_idx(len(ib), 2048, seed)]])
    return synth.sample_idx(n, 4096, seed=seed)


def synth_sample(n, workload):
    import synth
    return synth.sample_idx(n, 4096, seed=SAMPLE_SEED.get(workload, 100))


# ------------------------------------------------------------------ main


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="cube16m", choices=sorted(WORKLOADS))
    ap.add_argument("--mode", default="", choices=["", "plain", "quad", "learned"],
                    help="force evaluated per step (default: learned for the cube, plain otherwise)")
    ap.add_argument("--g-max", type=int, default=0)
    ap.add_argument("--group-mode", default="", choices=["", "chunk", "cell"])
    ap.add_argument("--chunk", type=int, default=0)
    ap.add_argument("--blocks-per-cu", type=int, default=0)
    ap.add_argument("--lpt", type=int, default=-1)
    ap.add_argument("--tile", type=int, default=0)
    ap.add_argument("--autotune", action="store_true",
                    help="sweep the schedule (of the corrected step in a corrected mode) and store the best in the cache")
    ap.add_argument("--autotune-reps", type=int, default=10, help="timed replays per autotuned schedule")
    ap.add_argument("--cache", default="", help="autotune cache file (default: the package's)")
    ap.add_argument("--no-learned", action="store_true", help="skip the learned-correction comparison on Plummer")
    ap.add_argument("--no-plummer", action="store_true", help="skip the Plummer 2^20 plain headline")
    ap.add_argument("--gate", type=float, default=0.4,
                    help="learned correction: the near-cell ratio l/|COM - c_g| (pairs near), or the layers' "
                         "l/n threshold (pairs all)")
    ap.add_argument("--near-ratio", type=float, default=0.0,
                    help="learned correction on near cells: the near ratio (0: the autotuned one, else the gate)")
    ap.add_argument("--err-target", type=float, default=0.0,
                    help="autotune of the learned step: the median force error the tuned step must hold "
                         "(0: the autotuner's default, 1e-3)")
    ap.add_argument("--pairs", default="near", choices=["near", "all"],
                    help="learned correction: network on the near cells only (walk lists them first; the far "
                         "cells stay monopoles), or on every cell (gated, textbook quadrupole below the gate)")
    ap.add_argument("--train-steps", type=int, default=3000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="after timing, one device-to-device copy of this many MiB (a known-size kernel for "
                         "calibrating hardware byte counters)")
    ap.add_argument("--quiet", action="store_true")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path (run with --gpus 1)",
              file=sys.stderr)
        sys.exit(2)

    def log(*a):
        if not args.quiet:
            print(*a, file=sys.stderr, flush=True)

    import torch
    import paper_1206_1199_amd as otoo
    from paper_1206_1199_amd import autotune as at

    mode = args.mode or HEADLINE_MODE.get(args.workload, "plain")
    pos, m, eps, theta, desc, classes = make_workload(args.workload)
    log(f"workload {desc}: n={len(m)}, {mode} force")
    t0 = time.perf_counter()
    with marker("tree build"):
        tree = otoo.Tree(pos, m, n_crit=16)
    t1 = time.perf_counter()
    del pos
    ctx = otoo.Context(0)

    near = args.pairs == "near"
    near_ratio = args.gate if (mode == "learned" and near) else 0.0
    perm, pos32, mass32, cm = tree.export(4 if mode == "plain" else 12)
    sample = workload_sample(args.workload, classes, perm, len(m))
    net, training, params = None, None, None
    if mode == "learned":
        net, training = train_network(ctx, log, args.train_steps, gate=args.gate, near=near)
        params = net.get_params()[0]

    sched_mode = mode if (mode != "learned" or near) else "learned-all"
    key = at.cache_key(args.workload, sched_mode)
    cache_path = args.cache or at.DEFAULT_CACHE
    if args.autotune:
        grid = dict(at.GRID)
        if args.workload in GROUPS:
            grid["group"] = GROUPS[args.workload]
        kind = {"plain": -1, "quad": otoo.CORR_QUAD, "learned": otoo.CORR_MLP}[mode]
        if mode == "learned" and near:
            # the near ratio is tuned with the schedule, under a bound on the step's median error
            # at the accuracy sample (FP64 direct sums on the device)
            ref = types.SimpleNamespace(pos=torch.from_numpy(pos32).to("cuda:0"),
                                        mass=torch.from_numpy(mass32).to("cuda:0"))
            a_ref, _ = direct_reference(ctx, ref, sample, eps)
            del ref
            ratios = (args.near_ratio,) if args.near_ratio > 0 else at.NEAR_RATIOS
            best, table = at.autotune_learned(tree, eps, theta, ctx, net, sample, a_ref, ratios=ratios,
                                              err_target=args.err_target or at.ERR_TARGET, grid=grid,
                                              reps=args.autotune_reps, log=log)
            near_ratio = best["near_ratio"]
        else:
            best, table = at.autotune(tree, eps, theta, ctx, grid=grid, log=log, corr_kind=kind, net=net,
                                      reps=args.autotune_reps, near_ratio=near_ratio)
        at.save_cache(key, best, cache_path)
        sched = {k: best[k] for k in at.DEFAULT_SCHEDULE}
        source = "autotuned now" + ("" if mode == "plain" else f" ({mode} step)")
    else:
        sched, source = at.cached_schedule(args.workload, 0, cache_path, mode=sched_mode)
        if mode == "learned" and near:
            near_ratio = at.cached_near_ratio(args.workload, 0, cache_path, default=near_ratio)
    if mode == "learned" and near and args.near_ratio > 0:
        near_ratio = args.near_ratio
    for k, v in (("g_max", args.g_max), ("group_mode", args.group_mode), ("chunk", args.chunk),
                 ("blocks_per_cu", args.blocks_per_cu), ("tile", args.tile)):
        if v:
            sched[k] = v
            source += "+override"
    if args.lpt >= 0:
        sched["lpt"] = args.lpt
    gmode = otoo.GROUP_CHUNK if sched["group_mode"] == "chunk" else otoo.GROUP_CELL
    log(f"schedule ({source}): {sched}" + (f", near ratio {near_ratio}" if near_ratio > 0 else ""))

    t2 = time.perf_counter()
    with marker("host walk"):
        lists = tree.walk(theta=theta, g_max=sched["g_max"], group_mode=gmode, near_ratio=near_ratio)
    t3 = time.perf_counter()
    log(f"tree {1e3 * (t1 - t0):.0f} ms, walk {1e3 * (t3 - t2):.0f} ms: groups {lists.n_groups}, "
        f"entries {lists.n_entries}, interactions {lists.interactions}, cell pairs {int(lists.pair_off[-1])}")

    torch.cuda.synchronize()
    t4 = time.perf_counter()
    with marker("copy to device"):
        d = otoo.DeviceLists.from_host(pos32, mass32, lists, cm, "cuda:0")
        torch.cuda.synchronize()
    t5 = time.perf_counter()

    ctx.set_tuning(chunk=sched["chunk"], blocks_per_cu=sched["blocks_per_cu"], lpt=sched["lpt"], tile=sched["tile"])
    out = ctx.outputs(d.n)
    gc = torch.empty((d.n_groups, otoo.CORR_STRIDE), dtype=torch.float32, device="cuda:0")
    reps = max(5, min(args.steps, 20))
    step = make_step(ctx, d, eps, mode, net, out, gc)
    ms, wall_ms = time_graph(ctx, step, args.warmup, args.steps)
    k_ms = graph_kernel_ms(ctx, step, reps)
    k_src = f"HIP events around k_force captured in the step's graph, mean of {reps} replays"
    if k_ms is None:
        k_ms, _ = kernel_times(ctx, d, eps, mode, net, out, gc, reps)
        k_src = f"HIP events around k_force, mean of {reps} eager calls"
    corr_ms = 0.0
    if mode != "plain":   # the step less the same force alone (its graph, same lists and correction input)
        force_ms, _ = time_graph(ctx, lambda: ctx.force(d, eps, out=out, gcorr=gc), args.warmup, args.steps)
        corr_ms = ms - force_ms
    log(f"force eval {ms:.3f} ms/step (wall {wall_ms:.3f}), force kernel {k_ms:.3f} ms, correction pass "
        f"{corr_ms:.3f} ms")

    acc = out[0].cpu().numpy().astype(np.float64)
    pot = out[1].cpu().numpy()
    inter = lists.interactions
    n_pairs = int(lists.pair_off[-1])
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
        "config": {"workload": desc, "correction": mode, "gate": args.gate if mode == "learned" else None,
                   "near_ratio": near_ratio if near_ratio > 0 else None,
                   "corrected_pairs": ("near" if near else "all") if mode == "learned" else
                   ("all" if mode == "quad" else None),
                   "n": int(len(m)), "groups": lists.n_groups, "list_entries": lists.n_entries,
                   "interactions": inter, "cell_pairs": n_pairs, "n_cells": tree.n_cells, "schedule": sched,
                   "schedule_source": source, "step": "correction pass + force in one captured graph"
                   if mode != "plain" else "force in one captured graph"},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP32_TFLOPS,
                     "traffic": measured_traffic(args.workload, mode, desc, sched),
                     "kernel": "k_force", "kernel_ms": k_ms, "kernel_ms_source": k_src,
                     "flops_per_interaction": FLOPS_PER_INTERACTION,
                     # the library is built with packed FP32 instructions disabled, which halves the issue ceiling
                     "peak_without_packed_fp32": PEAK_FP32_NONPACKED_TFLOPS,
                     "frac_without_packed_fp32": achieved / PEAK_FP32_NONPACKED_TFLOPS},
        "host": {"tree_build_ms": 1e3 * (t1 - t0), "walk_ms": 1e3 * (t3 - t2), "h2d_ms": 1e3 * (t5 - t4)},
        "step_breakdown": {"correction_pass_ms": corr_ms, "k_force_ms": k_ms, "graph_step_ms": ms,
                           "correction_pass_source": "step graph less a graph of the force alone"
                           if mode != "plain" else None},
    }
    if mode != "plain":
        res["roofline_correction"] = correction_roofline(corr_ms, n_pairs, mode)
    if training:
        res["training"] = training
    # accuracy of the tree force: FP64 direct sums on the device at a 4096-particle sample
    cls = {k: v[perm] for k, v in classes.items()}          # masks in device order
    a_dir, p_dir = direct_reference(ctx, d, sample, eps)
    et, ept = rel_err(acc[sample], a_dir), rel_err(pot[sample], p_dir)
    res["accuracy"] = {"tree_acc_median_vs_direct": float(np.median(et)),
                       "tree_acc_p99_vs_direct": float(np.quantile(et, 0.99)),
                       "tree_pot_median_vs_direct": float(np.median(ept)), "direct_sample": len(sample)}
    if mode != "plain":     # the same lists without the correction, for context
        ctx.force(d, eps, out=out)
        torch.cuda.synchronize()
        e0 = rel_err(out[0].cpu().numpy()[sample], a_dir)
        res["accuracy"]["plain_same_lists_acc_median_vs_direct"] = float(np.median(e0))
    for k, mask in cls.items():
        sel = mask[sample]
        res["accuracy"][f"tree_acc_median_vs_direct_{k}"] = float(np.median(et[sel])) if sel.any() else None
    log(f"accuracy {res['accuracy']}")
    if not args.no_cpu_baseline:
        if mode == "plain":
            base, (a_ref, p_ref), cpu_direct = cpu_baseline(pos32, mass32, lists, cm, eps, sample)
            ea, ep = rel_err(acc, a_ref), rel_err(pot, p_ref)
            res["cpu_baseline"] = base
            res["accuracy"].update({"parity_acc_median": float(np.median(ea)), "parity_acc_max": float(ea.max()),
                                    "parity_pot_median": float(np.median(ep)), "parity_pot_max": float(ep.max())})
            eda, edp = rel_err(a_dir, cpu_direct[0]), rel_err(p_dir, cpu_direct[1])
            res["accuracy"].update({"direct_parity_acc_max": float(eda.max()),
                                    "direct_parity_pot_max": float(edp.max())})
            for k, mask in cls.items():
                res["accuracy"][f"parity_acc_median_{k}"] = float(np.median(ea[mask]))
                res["accuracy"][f"parity_acc_max_{k}"] = float(ea[mask].max())
        else:
            # a bounded sample: every k-th group, k chosen for about 12 s of oracle work on 16 threads
            # (measured rates: about 6 us per (group, cell) pair for the FP64 network and its tensors,
            # 8e8 interactions/s for the list sums)
            est_s = 6e-6 * n_pairs + inter / 8e8
            step_g = int(min(max(1, np.ceil(est_s / 12.0)), max(1, lists.n_groups // 256)))
            groups = np.arange(0, lists.n_groups, step_g, dtype=np.int64)
            go = np.asarray(lists.group_off, np.int64)
            tgt = np.concatenate([np.arange(go[g], go[g + 1])[:4] for g in groups])
            base, (a_ref, p_ref) = cpu_baseline_corrected(pos32, mass32, lists, cm, eps, mode, params,
                                                          0.0 if near else args.gate, groups, tgt)
            res["cpu_baseline"] = base
            ea, ep = rel_err(acc[tgt], a_ref), rel_err(pot[tgt], p_ref)
            res["accuracy"].update({"parity_acc_median": float(np.median(ea)), "parity_acc_max": float(ea.max()),
                                    "parity_pot_median": float(np.median(ep)), "parity_pot_max": float(ep.max()),
                                    "parity_sample": len(tgt)})
        log(f"cpu baseline {res['cpu_baseline']['value']:.3f} Gint/s; parity {res['accuracy'].get('parity_acc_median')}")
    del d
    torch.cuda.empty_cache()
    if mode == "learned" and not args.no_learned:   # the same comparison on the benchmark workload itself
        try:
            has_quad = at.cache_key(args.workload, "quad") in at.load_cache(cache_path)
            scheds = {"plain": at.cached_schedule(args.workload, 0, cache_path)[0],
                      "quad": at.cached_schedule(args.workload, 0, cache_path, mode="quad")[0] if has_quad else sched,
                      "learned": sched}
            # the step's own ratio, and 0.6, which holds the error bound to larger opening angles
            ratios = tuple(sorted({near_ratio, 0.6})) if near_ratio > 0 else (0.0,)
            res["learned_workload"] = workload_learned(ctx, net, training, log, tree, eps, theta, scheds, sample,
                                                       a_dir, reps, ratios)
        except Exception as e:  # the headline measurement stands on its own
            res["learned_workload"] = {"error": f"{type(e).__name__}: {e}"}
            log(f"workload comparison failed: {e}")
    if args.workload != "plummer1m" and not args.no_plummer:
        try:
            res["plummer1m"] = plain_headline(ctx, log, args.steps, args.warmup, reps)
        except Exception as e:  # the headline measurement stands on its own
            res["plummer1m"] = {"error": f"{type(e).__name__}: {e}"}
    if not args.no_learned:
        try:
            if net is None:
                net, training = train_network(ctx, log, args.train_steps, gate=args.gate, near=near)
            res["learned"] = learned_comparison(ctx, net, training, log, reps)
        except Exception as e:  # the headline measurement stands on its own
            res["learned"] = {"error": f"{type(e).__name__}: {e}"}
            log(f"learned comparison failed: {e}")
    if args.calib_copy_mib:
        nbytes = args.calib_copy_mib << 20
        src_t = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda:0")
        dst_t = torch.empty_like(src_t)
        torch.cuda.synchronize()
        dst_t.copy_(src_t)
        torch.cuda.synchronize()
        res["calib_copy_bytes"] = nbytes
    print(json.dumps(res), flush=True)


def correction_roofline(corr_ms, n_pairs, mode):
    """The correction pass against its bounds: the network's dense layers on
    the BF16 matrix cores (2 (32x64 + 64x64 + 64x6) flops per pair through the
    layers; the gate decides how many) and the FP32 expansion work (the
    quadrupole-form field and its two derivatives at the group centre, about
    300 flops per pair, counted for every pair)."""
    flops_exp = 300.0 * n_pairs
    return {"pass_ms": corr_ms, "pairs": n_pairs, "mode": mode,
            "expansion_tflops": flops_exp / (corr_ms * 1e-3) / 1e12 if corr_ms > 0 else None,
            "network_flops_per_gated_pair": 2 * (32 * 64 + 64 * 64 + 64 * 6), "bf16_mfma_peak_tflops": 2500.0}


if __name__ == "__main__":
    main()
