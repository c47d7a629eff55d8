"""FP64 CPU oracle of the octree gravity force path -- TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and the benchmark's CPU-baseline
leg may import this package.  It shares no code with the HIP library
(``paper_1206_1199_amd``) and imports nothing from it; both sides draw their
inputs from ``synth``.

Contents
  direct(pos, m, eps, tgt=None)           O(N^2) direct sum        (oracle.c)
  list_force(pos, m, lists, ..., tgt)     list sums, monopole cells
                                           (+ optional quadrupole-form
                                           tensors per (group, cell))  (oracle.c)
  point_field(x, src_off, src_idx, ...)   exact field of source sets at points
  quad_field(x, centre, quad, eps)        quadrupole-form field alone
  sph_kernel(r, h), sph_sum(pos, h, q)    SPH gather sums, brute force (oracle.c)
  tree                                    recursive octree, moments, walk (tree.py)
  mlp                                     FP64 network, loss and hand backward (mlp.py)

Pins: every function is checked in ``tests/test_oracle_*.py`` against closed
forms, invariants or brute force (see the test docstrings).  Nothing here is
"parity unpinned".
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile oracle.c with gcc (-O2, OpenMP, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        I = ctypes.c_int64
        D = ctypes.c_double
        lib.oracle_direct.argtypes = [I, P, P, D, I, P, P, P]
        lib.oracle_direct.restype = None
        lib.oracle_list_force.argtypes = [I, P, P, I, P, P, P, I, P, P, P, P, P, D, I, P, P, P]
        lib.oracle_list_force.restype = ctypes.c_int
        lib.oracle_point_field.argtypes = [I, P, P, P, P, P, D, P, P]
        lib.oracle_point_field.restype = None
        lib.oracle_quad_field.argtypes = [I, P, P, P, D, P, P]
        lib.oracle_quad_field.restype = None
        lib.oracle_list_force_expanded.argtypes = [I, P, P, I, P, P, P, I, P, P, P, P, P, D, I, P, P, P]
        lib.oracle_list_force_expanded.restype = ctypes.c_int
        lib.oracle_quad_derivs.argtypes = [I, P, P, P, D, P, P, P, P]
        lib.oracle_quad_derivs.restype = None
        lib.oracle_sph_kernel.argtypes = [D, D]
        lib.oracle_sph_kernel.restype = D
        lib.oracle_sph_sum.argtypes = [I, P, P, P, I, P, P]
        lib.oracle_sph_sum.restype = None
        _lib = lib
    return _lib


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _i64(a):
    return np.ascontiguousarray(a, dtype=np.int64)


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def direct(pos, mass, eps, tgt=None):
    """Direct sum over all j != i.  Returns (acc[T,3], pot[T]) for targets tgt (default all)."""
    lib = _load()
    pos = _f64(pos)
    mass = _f64(mass)
    n = len(mass)
    tg = None if tgt is None else _i64(tgt)
    nt = n if tg is None else len(tg)
    acc = np.empty((nt, 3))
    pot = np.empty(nt)
    lib.oracle_direct(n, _ptr(pos), _ptr(mass), float(eps), nt, _ptr(tg), _ptr(acc), _ptr(pot))
    return acc, pot


def list_force(pos, mass, group_off, list_off, list_idx, cell_com, cell_mass, eps,
               tgt=None, n_cellent=None, quad=None, expanded=False):
    """Interaction-list sums (see oracle.c).  Returns (acc[T,3], pot[T]).

    With ``quad`` (one tensor per (group, cell) pair: the first
    ``n_cellent[g]`` entries of each group's list, which must be cells) those
    cells also act through the quadrupole form, per target
    (``expanded=False``) or through a second-order local expansion about the
    group's box centre (``expanded=True``); later cell entries act as
    monopoles only.
    """
    lib = _load()
    pos = _f64(pos)
    mass = _f64(mass)
    n = len(mass)
    go = _i64(group_off)
    lo = _i64(list_off)
    li = _i64(list_idx)
    cc = _f64(cell_com).reshape(-1, 3)
    cm = _f64(cell_mass)
    tg = None if tgt is None else _i64(tgt)
    nt = n if tg is None else len(tg)
    nce = po = qd = None
    if quad is not None:
        nce = _i64(n_cellent)
        po = _i64(np.concatenate([[0], np.cumsum(nce)]))
        qd = _f64(quad).reshape(-1, 6)
        if len(qd) != po[-1]:
            raise ValueError("quad must hold one tensor per (group, cell) pair")
    acc = np.empty((nt, 3))
    pot = np.empty(nt)
    fn = lib.oracle_list_force_expanded if (expanded and quad is not None) else lib.oracle_list_force
    rc = fn(n, _ptr(pos), _ptr(mass), len(go) - 1, _ptr(go), _ptr(lo), _ptr(li),
            len(cm), _ptr(cc), _ptr(cm), _ptr(nce), _ptr(po), _ptr(qd),
            float(eps), nt, _ptr(tg), _ptr(acc), _ptr(pot))
    if rc != 0:
        raise ValueError("list entry out of range or cell/particle order violated")
    return acc, pot


def point_field(x, src_off, src_idx, pos, mass, eps):
    """Exact softened field at points x[T,3] of source sets given as a CSR over particles."""
    lib = _load()
    x = _f64(x).reshape(-1, 3)
    so = _i64(src_off)
    si = _i64(src_idx)
    pos = _f64(pos)
    mass = _f64(mass)
    acc = np.empty((len(x), 3))
    pot = np.empty(len(x))
    lib.oracle_point_field(len(x), _ptr(x), _ptr(so), _ptr(si), _ptr(pos), _ptr(mass), float(eps),
                           _ptr(acc), _ptr(pot))
    return acc, pot


def quad_field(x, centre, quad, eps):
    """Quadrupole-form field alone at points x[T,3] of tensors quad[T,6] centred at centre[T,3]."""
    lib = _load()
    x = _f64(x).reshape(-1, 3)
    c = _f64(centre).reshape(-1, 3)
    q = _f64(quad).reshape(-1, 6)
    acc = np.empty((len(x), 3))
    pot = np.empty(len(x))
    lib.oracle_quad_field(len(x), _ptr(x), _ptr(c), _ptr(q), float(eps), _ptr(acc), _ptr(pot))
    return acc, pot


def quad_derivs(x, centre, quad, eps):
    """Quadrupole-form field, Jacobian [T,6] (xx,yy,zz,xy,xz,yz), Hessian [T,10]
    (xxx,yyy,zzz,xxy,xxz,xyy,yyz,xzz,yzz,xyz) and potential at points."""
    lib = _load()
    x = _f64(x).reshape(-1, 3)
    c = _f64(centre).reshape(-1, 3)
    q = _f64(quad).reshape(-1, 6)
    acc = np.empty((len(x), 3))
    jac = np.empty((len(x), 6))
    hess = np.empty((len(x), 10))
    pot = np.empty(len(x))
    lib.oracle_quad_derivs(len(x), _ptr(x), _ptr(c), _ptr(q), float(eps), _ptr(acc), _ptr(jac), _ptr(hess),
                           _ptr(pot))
    return acc, jac, hess, pot


def sph_kernel(r, h):
    """Cubic B-spline W(r, h) of compact support h (oracle.c, sph_w)."""
    lib = _load()
    return float(lib.oracle_sph_kernel(float(r), float(h)))


def sph_sum(pos, h, q, tgt=None):
    """s_i = sum_j q_j (W(r_ij, h_i) + W(r_ij, h_j)) / 2 over all j, self included."""
    lib = _load()
    pos, h, q = _f64(pos), _f64(h), _f64(q)
    n = len(h)
    tg = None if tgt is None else _i64(tgt)
    nt = n if tg is None else len(tg)
    out = np.empty(nt)
    lib.oracle_sph_sum(n, _ptr(pos), _ptr(h), _ptr(q), nt, _ptr(tg), _ptr(out))
    return out


def rel_err(a, ref):
    """Per-row relative error |a - ref| / |ref| (vectors) or |a - ref|/|ref| (scalars)."""
    a = np.asarray(a, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    if a.ndim == 2:
        return np.linalg.norm(a - ref, axis=1) / np.linalg.norm(ref, axis=1)
    return np.abs(a - ref) / np.abs(ref)
