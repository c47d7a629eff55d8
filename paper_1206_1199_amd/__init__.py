"""MI355X octree gravity force library: thin Python binding over libotoo.so.

Argument marshalling only.  The tree build and walk run in the library's
C++/OpenMP host code; every step of the force evaluation runs in its HIP
kernels.  PyTorch supplies device memory and streams.  There is no fallback:
if ``libotoo.so`` is missing, importing the binding's entry points raises.

    tree  = Tree(pos64, mass64, n_crit=16)          # host octree (key order)
    lists = tree.walk(theta=0.5, g_max=64)          # interaction-list CSR
    perm, pos32, mass32, cell_mom = tree.export(4)
    dev   = DeviceLists.from_host(pos32, mass32, lists, cell_mom, "cuda:0")
    ctx   = Context(device=0)
    acc, pot = ctx.force(dev, eps=0.01)

Environment overrides: OTOO_CHUNK, OTOO_TILE, OTOO_BLOCKS_PER_CU, OTOO_LPT and
OTOO_DEBUG_VALIDATE set the schedule of every new Context; OTOO_GMAX sets the
walks' default group size (64 otherwise); OTOO_AUTOTUNE_CACHE names the
autotuner's cache file.
"""
from __future__ import annotations

import ctypes
import math
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libotoo.so")

OK, EINVAL, ENOMEM, EHIP, EUNSUPPORTED = 0, -1, -2, -3, -4
MAX_GROUP = 256
THETA_LIMIT = 1.15
MAC_BH, MAC_ABSOLUTE = 0, 1
GROUP_CHUNK, GROUP_CELL = 0, 1
NOALLOC_SCRATCH_BYTES = 128 * 1024 * 1024   # OTOO_NOALLOC_SCRATCH_BYTES: otoo_force_noalloc's array per GPU
CORR_PAIRS, CORR_QUAD, CORR_MLP = 0, 1, 2
CORR_STRIDE = 24

_lib = None

_ENV_KEYS = (("OTOO_CHUNK", "chunk"), ("OTOO_TILE", "tile"), ("OTOO_BLOCKS_PER_CU", "blocks_per_cu"),
             ("OTOO_LPT", "lpt"), ("OTOO_DEBUG_VALIDATE", "debug_validate"), ("OTOO_GMAX", "g_max"))


def env_overrides(environ=None) -> dict:
    """Integer settings from the environment (the OTOO_* variables above), by
    field name; unset or empty variables are left out."""
    env = os.environ if environ is None else environ
    out = {}
    for key, name in _ENV_KEYS:
        v = env.get(key, "")
        if v.strip():
            try:
                out[name] = int(v)
            except ValueError:
                raise ValueError(f"{key}={v!r} is not an integer") from None
    return out


def _g_max(g_max):
    return int(g_max) if g_max is not None else env_overrides().get("g_max", 64)


class OtooError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"otoo error {code}: {msg}")
        self.code = code


class _WalkParams(ctypes.Structure):
    _fields_ = [("mac", ctypes.c_int32), ("theta", ctypes.c_double), ("delta", ctypes.c_double),
                ("m_limit", ctypes.c_double), ("group_mode", ctypes.c_int32), ("g_max", ctypes.c_int32),
                ("near_ratio", ctypes.c_double)]


class _Lists(ctypes.Structure):
    _fields_ = [("n_groups", ctypes.c_int32), ("n_entries", ctypes.c_int64), ("interactions", ctypes.c_int64),
                ("group_off", ctypes.POINTER(ctypes.c_int32)), ("list_off", ctypes.POINTER(ctypes.c_int64)),
                ("list_idx", ctypes.POINTER(ctypes.c_int32)), ("n_cellent", ctypes.POINTER(ctypes.c_int32)),
                ("group_box", ctypes.POINTER(ctypes.c_float)), ("n_near", ctypes.POINTER(ctypes.c_int32)),
                ("impl", ctypes.c_void_p)]


class Tuning(ctypes.Structure):
    _fields_ = [("chunk", ctypes.c_int32), ("blocks_per_cu", ctypes.c_int32), ("lpt", ctypes.c_int32),
                ("debug_validate", ctypes.c_int32), ("tile", ctypes.c_int32), ("net_kernel", ctypes.c_int32),
                ("corr_chunks", ctypes.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class GroupChoice(ctypes.Structure):
    _fields_ = [("group_mode", ctypes.c_int32), ("g_max", ctypes.c_int32)]


EXPORTED = [
    "otoo_tree_build", "otoo_tree_free", "otoo_tree_info", "otoo_tree_export", "otoo_tree_cells",
    "otoo_tree_links", "otoo_tree_walk", "otoo_tree_groups", "otoo_tree_walk_range", "otoo_tree_walk_sph", "otoo_lists_free", "otoo_create", "otoo_destroy",
    "otoo_set_stream", "otoo_last_error", "otoo_set_tuning", "otoo_get_tuning", "otoo_force", "otoo_force_noalloc",
    "otoo_check", "otoo_enable_timing", "otoo_last_timing", "otoo_graph_capture", "otoo_graph_launch",
    "otoo_autotune", "otoo_autotune_step", "otoo_set_scratch_limit", "otoo_force_plan", "otoo_group_layout",
    "otoo_scratch_generation",
    "otoo_quad_exact", "otoo_correction", "otoo_direct", "otoo_sph_sum", "otoo_mlp_num_params", "otoo_mlp_create", "otoo_mlp_destroy", "otoo_mlp_set_params", "otoo_mlp_set_gate",
    "otoo_mlp_get_params", "otoo_mlp_save", "otoo_mlp_load", "otoo_mlp_forward", "otoo_mlp_infer",
    "otoo_mlp_train_samples", "otoo_mlp_sample_weights", "otoo_mlp_backward", "otoo_mlp_train_step",
]


def lib():
    """Load libotoo.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_1206_1199_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    P, I32, I64, D, F = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_float
    pp = ctypes.POINTER(ctypes.c_void_p)
    sig = {
        "otoo_tree_build": ([P, P, I64, I32, pp], I32),
        "otoo_tree_free": ([P], None),
        "otoo_tree_info": ([P, P, P, P, P, P], I32),
        "otoo_tree_export": ([P, P, P, P, P, I32], I32),
        "otoo_tree_cells": ([P, P, P, P, P, P, P, P, P, P, P], I32),
        "otoo_tree_links": ([P, P, P], I32),
        "otoo_tree_walk": ([P, ctypes.POINTER(_WalkParams), ctypes.POINTER(ctypes.POINTER(_Lists))], I32),
        "otoo_tree_walk_sph": ([P, P, I32, I32, ctypes.POINTER(ctypes.POINTER(_Lists))], I32),
        "otoo_tree_groups": ([P, I32, I32, ctypes.POINTER(I32)], I32),
        "otoo_tree_walk_range": ([P, ctypes.POINTER(_WalkParams), I32, I32,
                                  ctypes.POINTER(ctypes.POINTER(_Lists))], I32),
        "otoo_lists_free": ([ctypes.POINTER(_Lists)], None),
        "otoo_create": ([pp, I32], I32),
        "otoo_destroy": ([P], I32),
        "otoo_set_stream": ([P, P], I32),
        "otoo_last_error": ([P], ctypes.c_char_p),
        "otoo_set_tuning": ([P, ctypes.POINTER(Tuning)], I32),
        "otoo_get_tuning": ([P, ctypes.POINTER(Tuning)], I32),
        "otoo_set_scratch_limit": ([P, I64], I32),
        "otoo_force_plan": ([I32, I32, I64, I32, I32, I32, ctypes.POINTER(I64)], I32),
        "otoo_group_layout": ([I32, I32, ctypes.POINTER(I32), ctypes.POINTER(I32)], I32),
        "otoo_scratch_generation": ([P, ctypes.POINTER(I64)], I32),
        "otoo_force": ([P, I32, P, P, I32, P, I64, P, P, I32, P, I32, F, P, P, P], I32),
        "otoo_force_noalloc": ([P, I32, P, P, I32, P, I64, P, P, I32, P, I32, F, P, P, P], I32),
        "otoo_correction": ([P, I32, P, I32, P, I32, P, P, I64, P, P, I64, P, I32, P, I32, F, P, P], I32),
        "otoo_quad_exact": ([P, I32, I32, I64, P, P, I64, P, I32, P, I32, P], I32),
        "otoo_direct": ([P, I32, P, P, I32, P, F, P, P], I32),
        "otoo_sph_sum": ([P, I32, P, P, P, I32, P, I64, P, P, P], I32),
        "otoo_check": ([P], I32),
        "otoo_enable_timing": ([P, I32], I32),
        "otoo_last_timing": ([P, ctypes.POINTER(F), ctypes.POINTER(F)], I32),
        "otoo_graph_capture": ([P, I32, P, P, I32, P, I64, P, P, I32, P, I32, F, P, P, P], I32),
        "otoo_graph_launch": ([P], I32),
        "otoo_autotune": ([P, P, ctypes.POINTER(_WalkParams), ctypes.POINTER(GroupChoice), I32,
                           ctypes.POINTER(Tuning), I32, F, I32, P, P, ctypes.POINTER(GroupChoice),
                           ctypes.POINTER(Tuning), ctypes.POINTER(F)], I32),
        "otoo_autotune_step": ([P, P, ctypes.POINTER(_WalkParams), ctypes.POINTER(GroupChoice), I32,
                                ctypes.POINTER(Tuning), I32, F, I32, P, I32, P, P, ctypes.POINTER(GroupChoice),
                                ctypes.POINTER(Tuning), ctypes.POINTER(F)], I32),
    }
    for name, (args, res) in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = res
    _lib = L
    return L


def _np_ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _check(rc, what="call"):
    if rc != OK:
        raise OtooError(rc, what)


# ------------------------------------------------------------------ host tree


@dataclass
class Lists:
    """Interaction-list CSR: host numpy arrays viewing the library's buffers,
    which are freed when the last of these arrays is gone."""
    group_off: np.ndarray    # int32 [G+1]
    list_off: np.ndarray     # int64 [G+1]
    list_idx: np.ndarray     # int32 [E]
    n_cellent: np.ndarray    # int32 [G]
    group_box: np.ndarray    # float32 [G, 6]
    interactions: int
    n_near: np.ndarray = None   # int32 [G]: the near cells listed first (walks with near_ratio > 0)
    near_ratio: float = 0.0

    @property
    def n_groups(self):
        return len(self.group_off) - 1

    @property
    def n_entries(self):
        return int(self.list_off[-1])

    @property
    def n_pair(self):
        """The (group, cell) pairs a cell correction covers, per group: the
        near cells when the walk split them, else every cell entry (each
        group's first entries)."""
        return self.n_near if self.near_ratio > 0 else self.n_cellent

    @property
    def pair_off(self):
        return np.concatenate([[0], np.cumsum(self.n_pair, dtype=np.int64)]).astype(np.int64)


class Tree:
    """Host octree (library-owned) of FP64 particles, sorted into key order."""

    def __init__(self, pos, mass, n_crit: int = 16):
        L = lib()
        pos = np.ascontiguousarray(pos, dtype=np.float64)
        mass = np.ascontiguousarray(mass, dtype=np.float64)
        if pos.ndim != 2 or pos.shape[1] != 3 or len(mass) != len(pos):
            raise ValueError("pos must be [n, 3] and mass [n]")
        h = ctypes.c_void_p()
        _check(L.otoo_tree_build(_np_ptr(pos), _np_ptr(mass), len(mass), int(n_crit), ctypes.byref(h)),
               "otoo_tree_build")
        self._h = h
        n = ctypes.c_int64()
        nc = ctypes.c_int64()
        depth = ctypes.c_int32()
        lo = (ctypes.c_double * 3)()
        side = ctypes.c_double()
        _check(L.otoo_tree_info(h, ctypes.byref(n), ctypes.byref(nc), ctypes.byref(depth), lo, ctypes.byref(side)))
        self.n, self.n_cells, self.depth = n.value, nc.value, depth.value
        self.root_lo = np.array(lo[:])
        self.root_side = side.value

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.otoo_tree_free(h)
            self._h = None

    def export(self, stride: int = 4):
        """(perm int64 [n], pos32 [n,3], mass32 [n], cell_mom float32 [n_cells, stride])."""
        perm = np.empty(self.n, np.int64)
        pos = np.empty((self.n, 3), np.float32)
        mass = np.empty(self.n, np.float32)
        cm = np.empty((self.n_cells, stride), np.float32)
        _check(lib().otoo_tree_export(self._h, _np_ptr(perm), _np_ptr(pos), _np_ptr(mass), _np_ptr(cm), stride),
               "otoo_tree_export")
        return perm, pos, mass, cm

    def cells(self):
        nc = self.n_cells
        out = dict(first=np.empty(nc, np.int64), count=np.empty(nc, np.int64), level=np.empty(nc, np.int32),
                   ijk=np.empty((nc, 3), np.int64), com=np.empty((nc, 3)), mass=np.empty(nc), side=np.empty(nc),
                   s=np.empty(nc), S6=np.empty((nc, 6)), bmax=np.empty(nc))
        _check(lib().otoo_tree_cells(self._h, *[_np_ptr(out[k]) for k in
                                               ("first", "count", "level", "ijk", "com", "mass", "side", "s",
                                                "S6", "bmax")]), "otoo_tree_cells")
        return out

    def links(self):
        m = self.n + self.n_cells
        nxt = np.empty(m, np.int64)
        more = np.empty(m, np.int64)
        _check(lib().otoo_tree_links(self._h, _np_ptr(nxt), _np_ptr(more)), "otoo_tree_links")
        return nxt, more

    def walk(self, theta: float = 0.5, g_max: int | None = None, group_mode: int = GROUP_CHUNK, mac: int = MAC_BH,
             delta: float = 0.01, m_limit: float = math.inf, near_ratio: float = 0.0) -> Lists:
        """Interaction lists; near_ratio > 0 lists each group's near cells
        (side >= near_ratio x distance of the COM from the group's box centre)
        first and makes them the lists' (group, cell) pairs."""
        p = _WalkParams(mac=mac, theta=theta, delta=delta, m_limit=m_limit, group_mode=group_mode,
                        g_max=_g_max(g_max), near_ratio=float(near_ratio))
        out = ctypes.POINTER(_Lists)()
        _check(lib().otoo_tree_walk(self._h, ctypes.byref(p), ctypes.byref(out)), "otoo_tree_walk")
        return self._take_lists(out, float(near_ratio))

    def n_groups(self, g_max: int | None = None, group_mode: int = GROUP_CHUNK) -> int:
        """Number of groups the walk forms for (group_mode, g_max)."""
        ng = ctypes.c_int32()
        _check(lib().otoo_tree_groups(self._h, int(group_mode), _g_max(g_max), ctypes.byref(ng)), "otoo_tree_groups")
        return ng.value

    def walk_range(self, g_begin: int, g_end: int, theta: float = 0.5, g_max: int | None = None,
                   group_mode: int = GROUP_CHUNK, mac: int = MAC_BH, delta: float = 0.01,
                   m_limit: float = math.inf) -> Lists:
        """The walk restricted to groups [g_begin, g_end): absolute group_off, list_off from 0."""
        p = _WalkParams(mac=mac, theta=theta, delta=delta, m_limit=m_limit, group_mode=group_mode,
                        g_max=_g_max(g_max))
        out = ctypes.POINTER(_Lists)()
        _check(lib().otoo_tree_walk_range(self._h, ctypes.byref(p), int(g_begin), int(g_end), ctypes.byref(out)),
               "otoo_tree_walk_range")
        return self._take_lists(out)

    def walk_sph(self, h, g_max: int | None = None, group_mode: int = GROUP_CHUNK) -> Lists:
        """Neighbour lists for SPH gather sums; h [n] in the caller's particle order."""
        h = np.ascontiguousarray(h, dtype=np.float64)
        if h.shape != (self.n,):
            raise ValueError("h must have one entry per particle")
        out = ctypes.POINTER(_Lists)()
        _check(lib().otoo_tree_walk_sph(self._h, h.ctypes.data_as(ctypes.c_void_p), int(group_mode), _g_max(g_max),
                                        ctypes.byref(out)), "otoo_tree_walk_sph")
        return self._take_lists(out)

    def _take_lists(self, out, near_ratio: float = 0.0) -> Lists:
        # the arrays are views of the library's buffers (no copy of the often
        # hundreds of MB of list indices); the buffers are freed with the last view
        owner = _ListsOwner(out)
        s = out.contents
        G, E = s.n_groups, s.n_entries
        return Lists(group_off=_view(s.group_off, ctypes.c_int32, G + 1, owner, np.int32),
                     list_off=_view(s.list_off, ctypes.c_int64, G + 1, owner, np.int64),
                     list_idx=_view(s.list_idx, ctypes.c_int32, E, owner, np.int32),
                     n_cellent=_view(s.n_cellent, ctypes.c_int32, G, owner, np.int32),
                     group_box=_view(s.group_box, ctypes.c_float, G * 6, owner, np.float32).reshape(G, 6),
                     interactions=int(s.interactions),
                     n_near=_view(s.n_near, ctypes.c_int32, G, owner, np.int32), near_ratio=near_ratio)


class _ListsOwner:
    """Holds a library list allocation until every array viewing it is gone."""

    def __init__(self, ptr):
        self.ptr = ptr

    def __del__(self):
        if _lib is not None and self.ptr is not None:
            _lib.otoo_lists_free(self.ptr)
            self.ptr = None


def _view(ptr, ctype, count, owner, dtype):
    if count == 0:
        return np.zeros(0, dtype)
    buf = (ctype * count).from_address(ctypes.cast(ptr, ctypes.c_void_p).value)
    buf._owner = owner
    return np.frombuffer(buf, dtype=dtype)


# ------------------------------------------------------------------ device


@dataclass
class DeviceLists:
    """Device-resident inputs of one force evaluation (torch tensors)."""
    pos: "object"        # float32 [n,3]
    mass: "object"       # float32 [n]
    group_off: "object"  # int32 [G+1]
    list_off: "object"   # int64 [G+1]
    list_idx: "object"   # int32 [E]
    cell_mom: "object"   # float32 [n_cells, stride]
    pair_off: "object"   # int64 [G+1]: prefix sums of the groups' cell counts
    n_entries: int
    interactions: int
    pair_count: int = -1   # pair_off[-1] known on the host (-1: read it from the device)
    group_box: "object" = None   # float32 [G, 6] lo xyz, hi xyz from the walk (None: found on the device)

    @property
    def n(self):
        return int(self.mass.shape[0])

    @property
    def n_groups(self):
        return int(self.group_off.shape[0]) - 1

    @property
    def n_cells(self):
        return int(self.cell_mom.shape[0])

    @property
    def n_pairs(self):
        # a host copy avoids a device read, which is not allowed inside a graph capture
        return self.pair_count if self.pair_count >= 0 else int(self.pair_off[-1].item())

    @classmethod
    def from_host(cls, pos32, mass32, lists: Lists, cell_mom, device="cuda:0"):
        import torch
        t = lambda a, dt: torch.from_numpy(np.ascontiguousarray(a, dtype=dt)).to(device)
        cm = cell_mom if len(cell_mom) else np.zeros((1, cell_mom.shape[1]), np.float32)
        return cls(pos=t(pos32, np.float32), mass=t(mass32, np.float32), group_off=t(lists.group_off, np.int32),
                   list_off=t(lists.list_off, np.int64),
                   list_idx=t(lists.list_idx if lists.n_entries else np.zeros(1, np.int32), np.int32),
                   cell_mom=t(cm, np.float32)[:len(cell_mom)], pair_off=t(lists.pair_off, np.int64),
                   n_entries=lists.n_entries, interactions=lists.interactions, pair_count=int(lists.pair_off[-1]),
                   group_box=t(lists.group_box, np.float32))


def _lists_on_device(cls, pos, mass, cell_mom, lists: Lists):
    """DeviceLists of one batch: particle and cell arrays already on the device,
    the batch's CSR copied over (its group_off may start past particle 0)."""
    import torch
    dev = pos.device
    t = lambda a, dt: torch.from_numpy(np.ascontiguousarray(a, dtype=dt)).to(dev)
    return cls(pos=pos, mass=mass, group_off=t(lists.group_off, np.int32), list_off=t(lists.list_off, np.int64),
               list_idx=t(lists.list_idx if lists.n_entries else np.zeros(1, np.int32), np.int32),
               cell_mom=cell_mom, pair_off=t(lists.pair_off, np.int64), n_entries=lists.n_entries,
               interactions=lists.interactions, pair_count=int(lists.pair_off[-1]))


DeviceLists.on_device = classmethod(_lists_on_device)


def force_plan(n: int, n_groups: int, n_entries: int, n_cells: int, chunk: int, workgroups: int) -> int:
    """Scratch bytes of an otoo_force call with these sizes (host only, no
    device); raises OtooError(EINVAL) for sizes the call would refuse,
    among them work queues of 2^31 or more items."""
    b = ctypes.c_int64()
    rc = lib().otoo_force_plan(int(n), int(n_groups), int(n_entries), int(n_cells), int(chunk), int(workgroups),
                               ctypes.byref(b))
    _check(rc, "otoo_force_plan")
    return b.value


def group_layout(ng: int, tile: int):
    """The force kernel's lanes for a group of ng targets at tile depth
    ``tile`` (host only): (False, [256 // ng, 0, 0, 0]) for slices across the
    workgroup, or (True, [part sizes of the four waves])."""
    wp = ctypes.c_int32()
    parts = (ctypes.c_int32 * 4)()
    _check(lib().otoo_group_layout(int(ng), int(tile), ctypes.byref(wp), parts), "otoo_group_layout")
    return bool(wp.value), list(parts)


class CapturedGraph:
    """A torch CUDA graph of library calls on one context, guarded against
    replays after the context's scratch was allocated anew."""

    def __init__(self, ctx, graph, generation):
        self.ctx = ctx
        self.graph = graph
        self.generation = generation

    def stale(self) -> bool:
        return self.ctx.scratch_generation() != self.generation

    def replay(self):
        if self.stale():
            raise OtooError(EINVAL, "the context's scratch was reallocated after this graph was captured; "
                                    "capture it again")
        self.graph.replay()


def _tptr(x):
    return ctypes.c_void_p(x.data_ptr()) if x is not None else None


class Context:
    """One libotoo device context; work goes on torch's current stream of that device."""

    def __init__(self, device: int = 0):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("no HIP device visible: the force path has no CPU fallback")
        self.device = device
        h = ctypes.c_void_p()
        _check(lib().otoo_create(ctypes.byref(h), int(device)), "otoo_create")
        self._h = h
        self.sync_stream()
        sched = {k: v for k, v in env_overrides().items() if k != "g_max"}
        if sched:
            self.set_tuning(**sched)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.otoo_destroy(h)
            self._h = None

    def _raise(self, rc, what):
        if rc != OK:
            raise OtooError(rc, f"{what}: {lib().otoo_last_error(self._h).decode()}")

    def sync_stream(self):
        import torch
        s = torch.cuda.current_stream(self.device)
        self._raise(lib().otoo_set_stream(self._h, ctypes.c_void_p(s.cuda_stream)), "otoo_set_stream")

    def set_tuning(self, chunk=0, blocks_per_cu=0, lpt=None, debug_validate=None, tile=0, net_kernel=None,
                   corr_chunks=None):
        cur = self.tuning()
        t = Tuning(chunk=chunk, blocks_per_cu=blocks_per_cu, lpt=cur.lpt if lpt is None else int(lpt),
                   debug_validate=cur.debug_validate if debug_validate is None else int(debug_validate), tile=tile,
                   net_kernel=cur.net_kernel if net_kernel is None else int(net_kernel),
                   corr_chunks=cur.corr_chunks if corr_chunks is None else int(corr_chunks))
        self._raise(lib().otoo_set_tuning(self._h, ctypes.byref(t)), "otoo_set_tuning")

    def set_scratch_limit(self, max_bytes: int = 0):
        """Cap on each device scratch buffer of the context (0: no cap); a
        call that would need more raises OtooError(ENOMEM)."""
        self._raise(lib().otoo_set_scratch_limit(self._h, int(max_bytes)), "otoo_set_scratch_limit")

    def tuning(self) -> Tuning:
        t = Tuning()
        self._raise(lib().otoo_get_tuning(self._h, ctypes.byref(t)), "otoo_get_tuning")
        return t

    def _args(self, d: DeviceLists, eps, out_acc, out_pot, gcorr=None):
        stride = int(d.cell_mom.shape[1]) if d.cell_mom.dim() == 2 else 4
        return (self._h, d.n, _tptr(d.pos), _tptr(d.mass), d.n_groups, _tptr(d.group_off), int(d.n_entries),
                _tptr(d.list_off), _tptr(d.list_idx), d.n_cells, _tptr(d.cell_mom) if d.n_cells else None,
                stride, float(eps), _tptr(gcorr), _tptr(out_acc), _tptr(out_pot))

    def scratch_generation(self) -> int:
        """Counter raised whenever the context allocates a scratch buffer anew."""
        g = ctypes.c_int64()
        self._raise(lib().otoo_scratch_generation(self._h, ctypes.byref(g)), "otoo_scratch_generation")
        return g.value

    def capture(self, fn):
        """A replayable graph of fn() (calls on this context, with preallocated
        outputs).  fn runs once eagerly first, so that every scratch buffer is
        allocated outside the capture; the context follows the capture stream
        and returns to the current stream afterwards.  The graph names the
        context's scratch as it was at capture: ``replay`` raises once the
        context has allocated scratch anew (a later call needed more), instead
        of writing freed memory."""
        import torch
        fn()
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        try:
            with torch.cuda.graph(g):
                self.sync_stream()
                fn()
        finally:
            self.sync_stream()
        return CapturedGraph(self, g, self.scratch_generation())

    def outputs(self, n):
        import torch
        return (torch.empty((n, 3), dtype=torch.float32, device=f"cuda:{self.device}"),
                torch.empty(n, dtype=torch.float64, device=f"cuda:{self.device}"))

    def force(self, d: DeviceLists, eps: float, out=None, gcorr=None):
        """Accelerations [n,3] FP32 and potentials [n] FP64 in key order (asynchronous).

        ``gcorr``: optional per-group cell correction [n_groups, 24] from
        ``correction``.
        """
        acc, pot = out if out is not None else self.outputs(d.n)
        self._raise(lib().otoo_force(*self._args(d, eps, acc, pot, gcorr)), "otoo_force")
        return acc, pot

    def force_noalloc(self, d: DeviceLists, eps: float, out, gcorr=None):
        """otoo_force_noalloc: the force with the library's fixed per-GPU
        scratch array instead of the context's (no device allocation; the
        outputs ``out`` = (acc, pot) must be given)."""
        acc, pot = out
        self._raise(lib().otoo_force_noalloc(*self._args(d, eps, acc, pot, gcorr)), "otoo_force_noalloc")
        return acc, pot

    def correction(self, d: DeviceLists, kind: int, eps: float, net=None, corr=None, out=None):
        """Per-group correction expansion [n_groups, 24] (kind CORR_PAIRS with
        ``corr`` [n_pairs, 6], CORR_QUAD, or CORR_MLP with ``net``)."""
        import torch
        g = out if out is not None else torch.empty((d.n_groups, CORR_STRIDE), dtype=torch.float32,
                                                    device=f"cuda:{self.device}")
        self._raise(lib().otoo_correction(self._h, int(kind), net._h if net is not None else None, d.n, _tptr(d.pos),
                                          d.n_groups, _tptr(d.group_off), _tptr(d.group_box), int(d.n_entries),
                                          _tptr(d.list_off),
                                          _tptr(d.list_idx), d.n_pairs, _tptr(d.pair_off), d.n_cells,
                                          _tptr(d.cell_mom) if d.n_cells else None, int(d.cell_mom.shape[1]),
                                          float(eps), _tptr(corr), _tptr(g)), "otoo_correction")
        return g

    def quad_exact(self, d: DeviceLists, out=None):
        """Textbook quadrupole 3S - tr(S) I of each (group, cell) pair: float32 [n_pairs, 6]."""
        import torch
        if d.cell_mom.shape[1] != 12:
            raise ValueError("cell moments with stride 12 (second-moment tensor) are required")
        n_pairs = d.n_pairs
        corr = out if out is not None else torch.empty((max(n_pairs, 1), 6), dtype=torch.float32,
                                                       device=f"cuda:{self.device}")[:n_pairs]
        self._raise(lib().otoo_quad_exact(self._h, d.n, d.n_groups, int(d.n_entries), _tptr(d.list_off),
                                          _tptr(d.list_idx), n_pairs, _tptr(d.pair_off), d.n_cells,
                                          _tptr(d.cell_mom) if d.n_cells else None, int(d.cell_mom.shape[1]),
                                          _tptr(corr)),
                    "otoo_quad_exact")
        return corr

    def direct(self, pos, mass, tgt, eps: float):
        """FP64 direct sums at targets ``tgt`` (int32 device tensor of indices into
        ``pos``): (acc float64 [n_tgt, 3], pot float64 [n_tgt])."""
        import torch
        n_tgt = int(tgt.numel())
        dev = f"cuda:{self.device}"
        acc = torch.empty((max(n_tgt, 1), 3), dtype=torch.float64, device=dev)[:n_tgt]
        pot = torch.empty(max(n_tgt, 1), dtype=torch.float64, device=dev)[:n_tgt]
        self._raise(lib().otoo_direct(self._h, int(pos.shape[0]), _tptr(pos), _tptr(mass), n_tgt, _tptr(tgt),
                                      float(eps), _tptr(acc), _tptr(pot)), "otoo_direct")
        return acc, pot

    def sph_sum(self, d: DeviceLists, h, q, out=None):
        """SPH gather sums over the lists of ``d`` (from Tree.walk_sph): float32 [n].
        ``h`` and ``q`` are float32 device tensors in the device (key) order."""
        import torch
        o = out if out is not None else torch.empty(d.n, dtype=torch.float32, device=f"cuda:{self.device}")
        self._raise(lib().otoo_sph_sum(self._h, d.n, _tptr(d.pos), _tptr(h), _tptr(q), d.n_groups,
                                       _tptr(d.group_off), int(d.n_entries), _tptr(d.list_off), _tptr(d.list_idx),
                                       _tptr(o)), "otoo_sph_sum")
        return o

    def check(self):
        self._raise(lib().otoo_check(self._h), "otoo_check")

    def enable_timing(self, on=True):
        self._raise(lib().otoo_enable_timing(self._h, int(on)), "otoo_enable_timing")

    def last_timing(self):
        k = ctypes.c_float()
        t = ctypes.c_float()
        self._raise(lib().otoo_last_timing(self._h, ctypes.byref(k), ctypes.byref(t)), "otoo_last_timing")
        return k.value, t.value

    def graph_capture(self, d: DeviceLists, eps: float, out, gcorr=None):
        acc, pot = out
        self._raise(lib().otoo_graph_capture(*self._args(d, eps, acc, pot, gcorr)), "otoo_graph_capture")

    def graph_launch(self):
        self._raise(lib().otoo_graph_launch(self._h), "otoo_graph_launch")

    def autotune(self, tree: Tree, eps: float, choices, schedules, reps: int = 10, theta: float = 0.5,
                 mac: int = MAC_BH, delta: float = 0.01, m_limit: float = math.inf, corr_kind: int = -1, net=None,
                 near_ratio: float = 0.0):
        """Time every (group_mode, g_max) choice x device schedule as graph replays
        (otoo_autotune; with corr_kind CORR_QUAD or CORR_MLP (and ``net``)
        otoo_autotune_step, each replay being the correction pass and the
        force).  schedules: dicts with chunk, blocks_per_cu, lpt, tile.
        Returns (ms [n_choices, n_schedules], interactions [n_choices],
        best (group_mode, g_max), best Tuning, best ms).  Discards any graph the
        context held."""
        ch = (GroupChoice * len(choices))(*[GroupChoice(int(m), int(g)) for m, g in choices])
        sc = (Tuning * len(schedules))(*[Tuning(chunk=int(s["chunk"]), blocks_per_cu=int(s["blocks_per_cu"]),
                                                lpt=int(s["lpt"]), tile=int(s["tile"])) for s in schedules])
        ms = np.zeros((len(choices), len(schedules)), np.float32)
        inter = np.zeros(len(choices), np.int64)
        bc, bt, bms = GroupChoice(), Tuning(), ctypes.c_float()
        p = _WalkParams(mac=mac, theta=theta, delta=delta, m_limit=m_limit, group_mode=GROUP_CHUNK, g_max=1,
                        near_ratio=float(near_ratio))
        if corr_kind < 0:
            rc = lib().otoo_autotune(self._h, tree._h, ctypes.byref(p), ch, len(choices), sc, len(schedules),
                                     float(eps), int(reps), _np_ptr(ms), _np_ptr(inter), ctypes.byref(bc),
                                     ctypes.byref(bt), ctypes.byref(bms))
        else:
            rc = lib().otoo_autotune_step(self._h, tree._h, ctypes.byref(p), ch, len(choices), sc, len(schedules),
                                          float(eps), int(corr_kind), net._h if net is not None else None,
                                          int(reps), _np_ptr(ms), _np_ptr(inter), ctypes.byref(bc),
                                          ctypes.byref(bt), ctypes.byref(bms))
        self._raise(rc, "otoo_autotune")
        return ms, inter, (bc.group_mode, bc.g_max), bt, bms.value
