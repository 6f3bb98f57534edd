"""CPU oracle for the minimum spanning forest -- TEST INFRASTRUCTURE ONLY.

Nothing in the product path may import this package: only ``tests/``, the
smoke check in ``__graft_entry__.smoke`` and the CPU-baseline leg of
``bench.py`` use it.  It shares no code with the GPU library.

Contents (each restates the paper's definitions, Sec. II-B and II-C):

* ``kruskal``      plain C Kruskal + union-find over keys (w, edge id)
* ``check``        independent C certificate check (spanning forest + cycle
                   property by binary lifting)
* ``brute_force``  enumeration of all spanning forests (n <= 8)
* ``by_definition`` the O(m^2) definition: e is in the MSF iff its endpoints
                   differ and are not joined by lighter edges
* ``components``   number of connected components
* ``boruvka_rounds`` one plain Borůvka round at a time (Sec. II-C), giving the
                   live vertex and edge counts of every round
* ``filter_*``     the pieces of Filter-Borůvka (Sec. V, Alg. 2): pivot
                   sampling, light/heavy split and heavy-edge filtering
                   (filter_ref.py), and the same per-split trace from set
                   definitions (filter_def.py)
* ``features``     the pivot network's sample statistics (features.py)
* ``mlp_ref``      the pivot network in float64 (mlp_ref.py)
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

from .brute import brute_force, by_definition  # noqa: F401
from .rounds import boruvka_rounds  # noqa: F401

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

OK, EINVAL, ERANGE, ENOMEM = 0, -1, -2, -3


def build(force: bool = True) -> str:
    """Compile liboracle.so (gcc -O3, portable)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(
            ["gcc", "-O3", "-std=c11", "-fPIC", "-shared", "-Wall", "-Wextra",
             os.path.join(_HERE, "kruskal.c"), os.path.join(_HERE, "check.c"), "-o", tmp])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        lib = ctypes.CDLL(_LIB_PATH)
        vp, i64 = ctypes.c_void_p, ctypes.c_int64
        lib.oracle_msf_kruskal.argtypes = [vp, vp, vp, i64, i64, vp, vp, vp]
        lib.oracle_components.argtypes = [vp, vp, i64, i64]
        lib.oracle_components.restype = i64
        lib.oracle_sort_u64.argtypes = [vp, i64]
        lib.oracle_msf_check.argtypes = [vp, vp, vp, i64, i64, vp, vp, vp]
        _lib = lib
    return _lib


def _arr(u, v, w):
    u = np.ascontiguousarray(u, dtype=np.int32)
    v = np.ascontiguousarray(v, dtype=np.int32)
    w = np.ascontiguousarray(w, dtype=np.uint32)
    return u, v, w


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


class OracleError(RuntimeError):
    def __init__(self, status):
        super().__init__(f"oracle status {status}")
        self.status = status


def kruskal(u, v, w, n):
    """Returns (mask uint8[m], total weight, number of MSF edges)."""
    u, v, w = _arr(u, v, w)
    m = len(u)
    mask = np.zeros(max(m, 1), np.uint8)
    total = ctypes.c_uint64(0)
    count = ctypes.c_int64(0)
    st = _load().oracle_msf_kruskal(_p(u), _p(v), _p(w), m, n, _p(mask),
                                    ctypes.byref(total), ctypes.byref(count))
    if st != OK:
        raise OracleError(st)
    return mask[:m], int(total.value), int(count.value)


def check(u, v, w, n, mask):
    """Certificate check of a candidate mask: 0 = it is the MSF (see check.c)."""
    u, v, w = _arr(u, v, w)
    mask = np.ascontiguousarray(mask, dtype=np.uint8)
    total = ctypes.c_uint64(0)
    count = ctypes.c_int64(0)
    rc = _load().oracle_msf_check(_p(u), _p(v), _p(w), len(u), n, _p(mask),
                                  ctypes.byref(total), ctypes.byref(count))
    return rc, int(total.value), int(count.value)


def components(u, v, n):
    u = np.ascontiguousarray(u, dtype=np.int32)
    v = np.ascontiguousarray(v, dtype=np.int32)
    return int(_load().oracle_components(_p(u), _p(v), len(u), n))


def filter_boruvka(*args, **kwargs):
    """Filter-Borůvka step by step (see oracle/filter_ref.py)."""
    from .filter_ref import filter_boruvka as fb
    return fb(*args, **kwargs)


def sort_u64(a):
    a = np.ascontiguousarray(a, dtype=np.uint64).copy()
    st = _load().oracle_sort_u64(_p(a), len(a))
    if st != OK:
        raise OracleError(st)
    return a
