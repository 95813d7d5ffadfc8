"""ctypes wrapper around the oracle's C particle loop (particles.c).  Test infrastructure.

The shared object is built with gcc by ``build_oracle()`` (also called from the package's
build step); it is not part of the product library.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "particles.c")
_LIB = os.path.join(_HERE, "liboracle_particles.so")


def build_oracle(force=False):
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-std=c99", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Mesh(ctypes.Structure):
    _fields_ = [("n_tets", ctypes.c_int64), ("xyz", ctypes.c_void_p), ("tets", ctypes.c_void_p),
                ("tet_edges", ctypes.c_void_p), ("tet_faces", ctypes.c_void_p), ("nbr", ctypes.c_void_p),
                ("grad", ctypes.c_void_p)]


class PushStats(ctypes.Structure):
    _fields_ = [("n_crossings", ctypes.c_int64), ("max_crossings", ctypes.c_int64),
                ("n_absorbed", ctypes.c_int64), ("n_cap_exceeded", ctypes.c_int64)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = ctypes.CDLL(build_oracle())
        for name in ("orc_push", "orc_trace", "orc_deposit_path", "orc_gather", "orc_barycentric"):
            getattr(_lib, name).restype = ctypes.c_int if name in ("orc_push", "orc_trace", "orc_deposit_path") \
                else None
    return _lib


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


class CMesh:
    """Keeps contiguous copies of the oracle mesh arrays alive for the C code."""

    def __init__(self, mesh):
        self.mesh = mesh
        self.arrs = [np.ascontiguousarray(mesh.xyz, dtype=np.float64),
                     np.ascontiguousarray(mesh.tets, dtype=np.int64),
                     np.ascontiguousarray(mesh.tet_edges, dtype=np.int64),
                     np.ascontiguousarray(mesh.tet_faces, dtype=np.int64),
                     np.ascontiguousarray(mesh.nbr, dtype=np.int64),
                     np.ascontiguousarray(mesh.grad_lambda, dtype=np.float64)]
        self.s = _Mesh(mesh.n_tets, *[_p(a) for a in self.arrs])

    @property
    def ref(self):
        return ctypes.byref(self.s)


def push(cmesh, x, u, tet, alive, q, m, w, dt, e, b, dg, cap=64):
    """One particle step in place (x, u, tet, alive); current added to dg.
    Returns (status, PushStats)."""
    for a, dt_ in ((x, np.float64), (u, np.float64), (tet, np.int64), (alive, np.int8), (dg, np.float64)):
        assert a.dtype == dt_ and a.flags.c_contiguous
    e = np.ascontiguousarray(e, dtype=np.float64)
    b = np.ascontiguousarray(b, dtype=np.float64)
    st = PushStats()
    rc = lib().orc_push(cmesh.ref, ctypes.c_int64(len(tet)), _p(x), _p(u), _p(tet), _p(alive),
                        ctypes.c_double(q), ctypes.c_double(m), ctypes.c_double(w), ctypes.c_double(dt),
                        _p(e), _p(b), _p(dg), ctypes.c_int(cap), ctypes.byref(st))
    return rc, st


def trace(cmesh, t0, x0, d, cap=64, max_rec=256):
    """Follow x0 -> x0 + d from tet t0.  Returns (status, t_end, x_end, [(tet, point)...])."""
    x0 = np.ascontiguousarray(x0, dtype=np.float64)
    d = np.ascontiguousarray(d, dtype=np.float64)
    t_end = ctypes.c_int64()
    x_end = np.zeros(3)
    nc = ctypes.c_int64()
    rt = np.zeros(max_rec, dtype=np.int64)
    rp = np.zeros((max_rec, 3))
    st = lib().orc_trace(cmesh.ref, ctypes.c_int64(t0), _p(x0), _p(d), ctypes.c_int(cap), ctypes.byref(t_end),
                         _p(x_end), ctypes.byref(nc), _p(rt), _p(rp), ctypes.c_int64(max_rec))
    n = min(nc.value + (1 if st == 1 else 0), max_rec)
    return st, t_end.value, x_end, list(zip(rt[:n].tolist(), rp[:n]))


def deposit_path(cmesh, t0, x0, d, qw, dg, cap=64):
    x0 = np.ascontiguousarray(x0, dtype=np.float64)
    d = np.ascontiguousarray(d, dtype=np.float64)
    t_end = ctypes.c_int64()
    x_end = np.zeros(3)
    st = lib().orc_deposit_path(cmesh.ref, ctypes.c_int64(t0), _p(x0), _p(d), ctypes.c_double(qw), _p(dg),
                                ctypes.c_int(cap), ctypes.byref(t_end), _p(x_end))
    return st, t_end.value, x_end


def gather(cmesh, tet, x, e, b):
    tet = np.ascontiguousarray(tet, dtype=np.int64)
    x = np.ascontiguousarray(x, dtype=np.float64).reshape(-1, 3)
    E = np.zeros_like(x)
    B = np.zeros_like(x)
    lib().orc_gather(cmesh.ref, ctypes.c_int64(len(tet)), _p(tet), _p(x),
                     _p(np.ascontiguousarray(e, dtype=np.float64)), _p(np.ascontiguousarray(b, dtype=np.float64)),
                     _p(E), _p(B))
    return E, B


def boris(q, m, dt, E, B, u):
    """Single relativistic Boris update (returns the new u)."""
    E = np.ascontiguousarray(E, dtype=np.float64)
    B = np.ascontiguousarray(B, dtype=np.float64)
    uu = np.array(u, dtype=np.float64)
    f = lib().orc_boris
    f.restype = None
    f(ctypes.c_double(q), ctypes.c_double(m), ctypes.c_double(dt), _p(E), _p(B), _p(uu))
    return uu
