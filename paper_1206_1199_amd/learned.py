"""Learned cell correction: binding over libotoo's network entry points and the
training driver (data drawn from the method's own walks, trained on the GPU
by the library's forward/backward/Adam kernels).

    net = Network(ctx)
    net.set_params(init_params(seed=0))
    X, aux, eps_all = make_training_set(ctx, net, configs, seed, gate=0.4)
    fit(net, X, aux, eps_all, steps=3000, batch=32768, lr=2e-3, seed=1)
    net.set_gate(0.4)
    gcorr = ctx.correction(dev_lists, CORR_MLP, eps, net=net)   # fused per-group expansion
    acc, pot = ctx.force(dev_lists, eps, gcorr=gcorr)
"""
from __future__ import annotations

import ctypes
import math
import time
from dataclasses import dataclass

import numpy as np

from . import DeviceLists, Lists, OtooError, Tree, _tptr, lib

N_PARAMS = 6662
N_IN = 32
AUX = 12


def _bind():
    L = lib()
    if getattr(L, "_mlp_bound", False):
        return L
    P, I32, I64, F = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_float
    pp = ctypes.POINTER(ctypes.c_void_p)
    sig = {
        "otoo_mlp_num_params": ([], I32),
        "otoo_mlp_create": ([P, pp], I32),
        "otoo_mlp_destroy": ([P], I32),
        "otoo_mlp_set_params": ([P, P], I32),
        "otoo_mlp_set_gate": ([P, F], I32),
        "otoo_mlp_get_params": ([P, P, P, P, P], I32),
        "otoo_mlp_save": ([P, ctypes.c_char_p], I32),
        "otoo_mlp_load": ([P, ctypes.c_char_p], I32),
        "otoo_mlp_forward": ([P, P, I64, P], I32),
        "otoo_mlp_infer": ([P, I32, P, I32, P, I64, P, P, I64, P, I32, P, I32, F, P], I32),
        "otoo_mlp_train_samples": ([P, I32, P, P, I32, P, I64, P, P, I64, P, I32, P, I32, P, P, F, I64, P, P, P],
                                   I32),
        "otoo_mlp_sample_weights": ([P, I64, P, I32, P, P, P, F, P, ctypes.POINTER(I64)], I32),
        "otoo_mlp_backward": ([P, P, P, I64, F, P, P], I32),
        "otoo_mlp_train_step": ([P, P, P, I64, F, F, P], I32),
    }
    for name, (args, res) in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = res
    L._mlp_bound = True
    return L


def init_params(seed: int) -> np.ndarray:
    """He-uniform weights, zero biases, last layer scaled down (FP32 vector)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    parts = []
    for n_in, n_out, scale in ((32, 64, 1.0), (64, 64, 1.0), (64, 6, 0.1)):
        lim = math.sqrt(6.0 / n_in)
        parts.append(rng.uniform(-lim, lim, (n_in, n_out)).ravel() * scale)
        parts.append(np.zeros(n_out))
    p = np.concatenate(parts).astype(np.float32)
    assert p.size == N_PARAMS
    return p


class Network:
    """The correction network on one context's device and stream."""

    def __init__(self, ctx):
        L = _bind()
        assert L.otoo_mlp_num_params() == N_PARAMS
        self.ctx = ctx
        h = ctypes.c_void_p()
        ctx._raise(L.otoo_mlp_create(ctx._h, ctypes.byref(h)), "otoo_mlp_create")
        self._h = h
        self.gate = 0.0

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is None:
            return
        self._h = None
        try:
            _bind().otoo_mlp_destroy(h)   # safe after the context is gone
        except Exception:                 # interpreter shutdown: module globals already cleared
            pass

    def _raise(self, rc, what):
        self.ctx._raise(rc, what)

    def set_params(self, params):
        p = np.ascontiguousarray(params, dtype=np.float32)
        if p.size != N_PARAMS:
            raise ValueError(f"expected {N_PARAMS} parameters")
        self._raise(_bind().otoo_mlp_set_params(self._h, p.ctypes.data_as(ctypes.c_void_p)), "otoo_mlp_set_params")

    def set_gate(self, gate: float):
        """Run the layers only for pairs with BF16 feature l/n >= gate (textbook quadrupole elsewhere)."""
        self._raise(_bind().otoo_mlp_set_gate(self._h, float(gate)), "otoo_mlp_set_gate")
        self.gate = float(gate)

    def get_params(self):
        p = np.empty(N_PARAMS, np.float32)
        m = np.empty(N_PARAMS, np.float32)
        v = np.empty(N_PARAMS, np.float32)
        step = ctypes.c_int64()
        self._raise(_bind().otoo_mlp_get_params(self._h, p.ctypes.data_as(ctypes.c_void_p),
                                                m.ctypes.data_as(ctypes.c_void_p),
                                                v.ctypes.data_as(ctypes.c_void_p), ctypes.byref(step)),
                    "otoo_mlp_get_params")
        return p, m, v, step.value

    def save(self, path):
        self._raise(_bind().otoo_mlp_save(self._h, str(path).encode()), "otoo_mlp_save")

    def load(self, path):
        self._raise(_bind().otoo_mlp_load(self._h, str(path).encode()), "otoo_mlp_load")

    def forward(self, X):
        """Raw outputs [rows, 6] for BF16 features X (int16 tensor [rows, 32])."""
        import torch
        out = torch.empty((X.shape[0], 6), dtype=torch.float32, device=X.device)
        self._raise(_bind().otoo_mlp_forward(self._h, _tptr(X), int(X.shape[0]), _tptr(out)), "otoo_mlp_forward")
        return out

    def infer(self, d: DeviceLists, eps: float, out=None):
        """Learned tensors [n_pairs, 6] for otoo_force (d.cell_mom must have stride 12)."""
        import torch
        n_pairs = d.n_pairs
        corr = out if out is not None else torch.empty((max(n_pairs, 1), 6), dtype=torch.float32,
                                                       device=d.pos.device)[:n_pairs]
        self._raise(_bind().otoo_mlp_infer(self._h, d.n, _tptr(d.pos), d.n_groups, _tptr(d.group_off),
                                           int(d.n_entries), _tptr(d.list_off), _tptr(d.list_idx), n_pairs,
                                           _tptr(d.pair_off), d.n_cells, _tptr(d.cell_mom),
                                           int(d.cell_mom.shape[1]), float(eps), _tptr(corr)), "otoo_mlp_infer")
        return corr

    def train_samples(self, d: DeviceLists, cell_first, cell_count, eps: float, samples):
        """(X int16 [S, 32] BF16 bits, aux float32 [S, 12]) for samples int64 [S, 2] = (pair, particle)."""
        import torch
        S = int(samples.shape[0])
        X = torch.empty((max(S, 1), N_IN), dtype=torch.int16, device=d.pos.device)[:S]
        aux = torch.empty((max(S, 1), AUX), dtype=torch.float32, device=d.pos.device)[:S]
        self._raise(_bind().otoo_mlp_train_samples(
            self._h, d.n, _tptr(d.pos), _tptr(d.mass), d.n_groups, _tptr(d.group_off), int(d.n_entries),
            _tptr(d.list_off), _tptr(d.list_idx), d.n_pairs, _tptr(d.pair_off), d.n_cells, _tptr(d.cell_mom),
            int(d.cell_mom.shape[1]), _tptr(cell_first), _tptr(cell_count), float(eps), S, _tptr(samples),
            _tptr(X), _tptr(aux)), "otoo_mlp_train_samples")
        return X, aux

    def sample_weights(self, samples, acc, X, aux, gate: float = 0.0):
        """Training weights into aux[:, 10] (W / |a_i|^2, normalised over the
        kept samples) and the indices of the samples the gate keeps (int64
        device tensor, ascending); otoo_mlp_sample_weights."""
        import torch
        S = int(samples.shape[0])
        keep = torch.empty(max(S, 1), dtype=torch.int64, device=aux.device)
        n_keep = ctypes.c_int64()
        self._raise(_bind().otoo_mlp_sample_weights(self._h, S, _tptr(samples), int(acc.shape[0]), _tptr(acc),
                                                    _tptr(X), _tptr(aux), float(gate), _tptr(keep),
                                                    ctypes.byref(n_keep)), "otoo_mlp_sample_weights")
        return keep[:n_keep.value]

    def backward(self, X, aux, eps: float):
        """(gradient [6662] float32, loss) of the mean weighted loss over the samples."""
        g = np.empty(N_PARAMS, np.float32)
        loss = ctypes.c_float()
        self._raise(_bind().otoo_mlp_backward(self._h, _tptr(X), _tptr(aux), int(X.shape[0]), float(eps),
                                              g.ctypes.data_as(ctypes.c_void_p), ctypes.byref(loss)),
                    "otoo_mlp_backward")
        return g, loss.value

    def train_step(self, X, aux, eps: float, lr: float, want_loss: bool = True):
        loss = ctypes.c_float()
        self._raise(_bind().otoo_mlp_train_step(self._h, _tptr(X), _tptr(aux), int(X.shape[0]), float(eps),
                                                float(lr), ctypes.byref(loss) if want_loss else None),
                    "otoo_mlp_train_step")
        return loss.value if want_loss else None


# ------------------------------------------------------------------ training data


@dataclass
class SampleConfig:
    """One walk of a seeded workload contributing training samples."""
    workload: str          # "plummer", or "grf_cube" (n = ng^3 particles)
    n: int
    seed: int
    eps: float
    theta: float
    g_max: int = 64
    n_samples: int = 40000


def device_tree_arrays(tree: Tree, lists: Lists, device="cuda:0"):
    """DeviceLists with stride-12 cell moments plus each cell's particle range."""
    import torch
    _, pos32, mass32, cm = tree.export(12)
    d = DeviceLists.from_host(pos32, mass32, lists, cm, device)
    cells = tree.cells()
    first = torch.from_numpy(cells["first"].astype(np.int32)).to(device)
    count = torch.from_numpy(cells["count"].astype(np.int32)).to(device)
    return d, first, count


def draw_samples(lists: Lists, n_samples: int, rng: np.random.Generator) -> np.ndarray:
    """Uniform (pair, particle) draws: a random cell entry, a random target of its group."""
    pair_off = lists.pair_off
    n_pairs = int(pair_off[-1])
    if n_pairs == 0 or n_samples == 0:
        return np.zeros((0, 2), np.int64)
    p = rng.integers(0, n_pairs, n_samples)
    g = np.searchsorted(pair_off, p, side="right") - 1
    lo = lists.group_off[g].astype(np.int64)
    ng = (lists.group_off[g + 1] - lists.group_off[g]).astype(np.int64)
    i = lo + rng.integers(0, 1 << 62, n_samples) % ng
    return np.stack([p, i], axis=1).astype(np.int64)


def make_training_set(ctx, net: Network, configs, seed: int, device="cuda:0", log=None, gate: float = 0.0,
                      near: bool = False):
    """Training samples from seeded walks (exact cell sums computed on the GPU).

    The library weights each sample by 1 / |a_i|^2, a_i the total force on
    its target from the same walk (the per-particle relative error is what
    the correction is judged by), normalised so that the zero-correction loss
    of each configuration's kept samples is 1, and keeps only pairs the gate
    lets through to the layers (BF16 feature l/n >= gate); this function
    gathers the kept rows.  With near=True the walks list each group's near
    cells first (near_ratio = gate) and the samples are drawn from those
    pairs alone, all of them kept.  Returns (X int16 [S,32], aux float32
    [S,12], eps float32 [S]) on the device; samples of different softening
    lengths carry their own eps.
    """
    import torch
    import synth
    rng = np.random.Generator(np.random.PCG64(seed))
    Xs, auxs, epss = [], [], []
    for cfg in configs:
        t0 = time.perf_counter()
        if cfg.workload == "plummer":
            pos, m = synth.plummer(cfg.n, seed=cfg.seed)
        elif cfg.workload == "grf_cube":
            pos, m = synth.grf_cube(int(round(cfg.n ** (1.0 / 3.0))), seed=cfg.seed)
        else:
            raise ValueError(cfg.workload)
        tree = Tree(pos, m, n_crit=16)
        lists = tree.walk(theta=cfg.theta, g_max=cfg.g_max, near_ratio=gate if near else 0.0)
        d, first, count = device_tree_arrays(tree, lists, device)
        smp = torch.from_numpy(draw_samples(lists, cfg.n_samples, rng)).to(device)
        X, aux = net.train_samples(d, first, count, cfg.eps, smp)
        acc, _ = ctx.force(d, cfg.eps)          # the target's total (monopole-tree) force
        keep = net.sample_weights(smp, acc, X, aux, 0.0 if near else gate)
        X, aux = X[keep], aux[keep]
        Xs.append(X)
        auxs.append(aux)
        epss.append(torch.full((X.shape[0],), cfg.eps, dtype=torch.float32, device=device))
        if log:
            log(f"  samples from {cfg}: {X.shape[0]} in {time.perf_counter() - t0:.2f} s")
    torch.cuda.synchronize()
    ctx.check()
    return torch.cat(Xs), torch.cat(auxs), torch.cat(epss)


def fit(net: Network, X, aux, eps_all, steps: int, batch: int, lr: float, seed: int, X_val=None, aux_val=None,
        eps_val=None, log=None, log_every: int = 200):
    """Adam with a cosine learning-rate decay over `steps` minibatches.

    Samples of one batch share one softening length (batches are drawn within
    an eps class).  Returns the loss history [(step, train, val)].
    """
    import torch
    rng = np.random.Generator(np.random.PCG64(seed))
    classes = {}
    eps_host = eps_all.cpu().numpy()
    for e in np.unique(eps_host):
        classes[float(e)] = np.where(eps_host == e)[0]
    keys = sorted(classes)
    weights = np.array([len(classes[k]) for k in keys], float)
    weights /= weights.sum()
    hist = []
    for step in range(steps):
        e = keys[rng.choice(len(keys), p=weights)]
        idx = classes[e]
        sel = torch.from_numpy(np.sort(rng.choice(idx, size=min(batch, len(idx)), replace=False))).to(X.device)
        lr_t = lr * 0.5 * (1.0 + math.cos(math.pi * step / steps))
        want = log is not None and (step % log_every == 0 or step == steps - 1)
        loss = net.train_step(X[sel].contiguous(), aux[sel].contiguous(), e, lr_t, want_loss=want)
        if want:
            val = evaluate_loss(net, X_val, aux_val, eps_val) if X_val is not None else None
            hist.append((step, loss, val))
            log(f"  step {step}: train loss {loss:.4e}" + (f", validation {val:.4e}" if val is not None else ""))
    return hist


def evaluate_loss(net: Network, X, aux, eps_all):
    """Sample-weighted mean loss over eps classes (no update)."""
    import torch
    eps_host = eps_all.cpu().numpy()
    tot, cnt = 0.0, 0
    for e in np.unique(eps_host):
        idx = torch.from_numpy(np.where(eps_host == e)[0]).to(X.device)
        _, loss = net.backward(X[idx].contiguous(), aux[idx].contiguous(), float(e))
        tot += loss * len(idx)
        cnt += len(idx)
    return tot / max(cnt, 1)


def zero_correction_loss(aux):
    """The loss of the plain monopole (zero tensor) on these samples, mean w |t|^2,
    taken on the host (1 per configuration by the weights' normalisation)."""
    a = aux.cpu().numpy().astype(np.float64)
    return float(np.mean(a[:, 10] * (a[:, 6:9] ** 2).sum(axis=1)))
