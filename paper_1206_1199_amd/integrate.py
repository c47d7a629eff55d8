"""Gravity-only leap-frog loop around the device force evaluation.

The integration step of Sec. 5 restricted to gravity: (1) predict the
positions, (2) build the tree, (7) update the cell properties for gravity,
(8) walk and evaluate the force, (9) correct the velocities.  As in the
paper, everything except the force runs on the host: the state stays in FP64
on the host in the caller's particle order, the tree is rebuilt every step
and the force comes back from the device (kick-drift-kick leap-frog).

Two ways to run step (8):
- ``batches > 1``: the host walks the groups in batches on a worker thread
  while the device evaluates the batches already walked (the host rebuild
  overlapped with the GPU force);
- ``batches == 1``: one walk, then the step's force launch captured in a
  HIP graph and replayed (``use_graph``) or enqueued directly.
The forces are bitwise the same either way.
"""
from __future__ import annotations

import queue
import threading
import time
from dataclasses import dataclass, field

import numpy as np

from . import GROUP_CHUNK, Context, DeviceLists, Tree


@dataclass
class StepTimes:
    """Per-step host wall times: tree build, host walk (summed over batches),
    and step 8 as a whole (walk, copies and device force, overlapped when
    batched) until the forces are back on the host."""
    tree_ms: list = field(default_factory=list)
    walk_ms: list = field(default_factory=list)
    eval_ms: list = field(default_factory=list)


class LeapFrog:
    """Kick-drift-kick integrator with softening eps and opening angle theta."""

    def __init__(self, pos, vel, mass, eps: float, theta: float, g_max: int = 64, ctx: Context | None = None,
                 group_mode: int = GROUP_CHUNK, batches: int = 1, use_graph: bool = False):
        self.x = np.array(pos, dtype=np.float64)
        self.v = np.array(vel, dtype=np.float64)
        self.m = np.array(mass, dtype=np.float64)
        self.eps, self.theta, self.g_max, self.group_mode = eps, theta, g_max, group_mode
        self.batches, self.use_graph = max(1, int(batches)), use_graph
        self.ctx = ctx or Context(0)
        self.times = StepTimes()
        self.a, self.phi = self._force()

    def _walk_kw(self):
        return dict(theta=self.theta, g_max=self.g_max, group_mode=self.group_mode)

    def _evaluate_whole(self, tree, pos32, mass32, cm):
        import torch
        t0 = time.perf_counter()
        lists = tree.walk(**self._walk_kw())
        t1 = time.perf_counter()
        d = DeviceLists.from_host(pos32, mass32, lists, cm)
        out = self.ctx.outputs(d.n)
        if self.use_graph:
            self.ctx.graph_capture(d, self.eps, out)
            self.ctx.graph_launch()
        else:
            self.ctx.force(d, self.eps, out=out)
        torch.cuda.synchronize()
        return out, t1 - t0

    def _evaluate_pipelined(self, tree, pos32, mass32, cm):
        """Walk batches of groups on a worker thread; evaluate each on the
        device as soon as it is walked (the library call releases the GIL)."""
        import torch
        dev = f"cuda:{self.ctx.device}"
        pos_d = torch.from_numpy(pos32).to(dev)
        mass_d = torch.from_numpy(mass32).to(dev)
        cm_d = torch.from_numpy(np.ascontiguousarray(cm)).to(dev)
        G = tree.n_groups(self.g_max, self.group_mode)
        edges = np.linspace(0, G, min(self.batches, G) + 1).round().astype(int)
        ready: queue.Queue = queue.Queue()
        walk_s = [0.0]

        def walker():
            try:
                for b in range(len(edges) - 1):
                    t0 = time.perf_counter()
                    lists = tree.walk_range(int(edges[b]), int(edges[b + 1]), **self._walk_kw())
                    walk_s[0] += time.perf_counter() - t0
                    ready.put(lists)
            except BaseException as e:   # handed to the main thread
                ready.put(e)

        th = threading.Thread(target=walker, daemon=True)
        th.start()
        out = self.ctx.outputs(len(mass32))
        alive = []
        try:
            for _ in range(len(edges) - 1):
                lists = ready.get()
                if isinstance(lists, BaseException):
                    raise lists
                d = DeviceLists.on_device(pos_d, mass_d, cm_d, lists)
                self.ctx.force(d, self.eps, out=out)
                alive.append(d)        # keep each batch's device lists until the stream is done
            torch.cuda.synchronize()
        finally:
            th.join()
        return out, walk_s[0]

    def _force(self):
        t0 = time.perf_counter()
        tree = Tree(self.x, self.m, n_crit=16)                      # steps 2 and 7
        t1 = time.perf_counter()
        perm, pos32, mass32, cm = tree.export(4)
        if self.batches > 1:                                         # step 8
            (acc, pot), walk_s = self._evaluate_pipelined(tree, pos32, mass32, cm)
        else:
            (acc, pot), walk_s = self._evaluate_whole(tree, pos32, mass32, cm)
        a_k = acc.cpu().numpy().astype(np.float64)
        p_k = pot.cpu().numpy()
        t4 = time.perf_counter()
        self.ctx.check()
        a = np.empty_like(a_k)
        phi = np.empty_like(p_k)
        a[perm] = a_k
        phi[perm] = p_k
        for lst, dt in ((self.times.tree_ms, t1 - t0), (self.times.walk_ms, walk_s), (self.times.eval_ms, t4 - t1)):
            lst.append(1e3 * dt)
        return a, phi

    def step(self, dt: float):
        self.v += 0.5 * dt * self.a          # first half kick (closing step 9 of the previous step)
        self.x += dt * self.v                # step 1: drift / predict
        self.a, self.phi = self._force()     # steps 2, 7, 8
        self.v += 0.5 * dt * self.a          # step 9: correct

    def energy(self):
        """(kinetic, potential, total): K = 1/2 sum m v^2, W = 1/2 sum m phi."""
        k = 0.5 * float(np.sum(self.m * np.sum(self.v * self.v, axis=1)))
        w = 0.5 * float(np.sum(self.m * self.phi))
        return k, w, k + w

    def momentum(self):
        return np.sum(self.m[:, None] * self.v, axis=0)


def plummer_velocities(pos, seed: int, mass: float = 1.0):
    """Isotropic Plummer velocities (G = M = a = 1) by rejection sampling of
    q = v / v_esc from g(q) ~ q^2 (1 - q^2)^(7/2) (Aarseth, Henon & Wielen 1974)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    n = len(pos)
    r = np.linalg.norm(pos, axis=1)
    v_esc = np.sqrt(2.0 * mass) * (1.0 + r * r) ** -0.25
    q = np.empty(n)
    todo = np.arange(n)
    while len(todo):
        x = rng.uniform(0.0, 1.0, len(todo))
        y = rng.uniform(0.0, 0.1, len(todo))
        ok = y < x * x * (1.0 - x * x) ** 3.5
        q[todo[ok]] = x[ok]
        todo = todo[~ok]
    mu = rng.uniform(-1.0, 1.0, n)
    ph = rng.uniform(0.0, 2.0 * np.pi, n)
    s = np.sqrt(1.0 - mu * mu)
    dirs = np.stack([s * np.cos(ph), s * np.sin(ph), mu], axis=1)
    v = (q * v_esc)[:, None] * dirs
    return v - v.mean(axis=0)
