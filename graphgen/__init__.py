"""Seeded synthetic input graphs for the MSF library, its oracle and the bench.

This package only draws inputs; it contains none of the spanning-forest
arithmetic.  Arrays come back as numpy ``int32 u, int32 v, uint32 w`` (one
entry per undirected edge, edge id = index).  The C implementation in
``graphgen.c`` is multithreaded; ``graphgen.ref`` restates it in numpy for the
bit-exactness tests.

The families are the paper's (Sec. VII, "Instances and Methodology"): GNM,
RMAT with the Graph500 probabilities, 2D grid and 2D random geometric graphs.
``workload()`` returns the named configurations used by tests and the bench.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libgraphgen.so")
_lib = None

TAG_GNM, TAG_RMAT, TAG_PERM, TAG_RMAT_W, TAG_GRID_KEEP, TAG_GRID_W, TAG_RGG = 1, 2, 3, 4, 5, 6, 7
TAG_RGG3, TAG_RGG3_W, TAG_RHG, TAG_RHG_W = 9, 10, 11, 12


def build(force: bool = True) -> str:
    """Compile libgraphgen.so with gcc (portable -O3, no -march=native)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(
            ["gcc", "-O3", "-std=c11", "-ffp-contract=off", "-fPIC", "-shared", "-Wall", "-Wextra",
             os.path.join(_HERE, "graphgen.c"), "-o", tmp, "-lpthread", "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        lib = ctypes.CDLL(_LIB_PATH)
        i64, u32, u64, dbl, vp = (ctypes.c_int64, ctypes.c_uint32, ctypes.c_uint64,
                                  ctypes.c_double, ctypes.c_void_p)
        lib.gg_gnm.argtypes = [i64, i64, u32, u32, u64, vp, vp, vp]
        lib.gg_rmat.argtypes = [ctypes.c_int, i64, dbl, dbl, dbl, u32, u32, ctypes.c_int, u64,
                                vp, vp, vp]
        lib.gg_rmat_permute.argtypes = [ctypes.c_int, u64, vp, i64, vp]
        lib.gg_grid_build.argtypes = [i64, i64, dbl, ctypes.c_int, u32, u32, u64,
                                      ctypes.POINTER(i64)]
        lib.gg_grid_build.restype = vp
        lib.gg_rgg2d_build.argtypes = [i64, dbl, dbl, u64, ctypes.POINTER(i64)]
        lib.gg_rgg2d_build.restype = vp
        lib.gg_rgg3d_build.argtypes = [i64, dbl, u32, u32, u64, ctypes.POINTER(i64)]
        lib.gg_rgg3d_build.restype = vp
        lib.gg_rhg_build.argtypes = [i64, dbl, u32, u32, u64, ctypes.POINTER(i64)]
        lib.gg_rhg_build.restype = vp
        lib.gg_take.argtypes = [vp, vp, vp, vp]
        lib.gg_batch_plan.argtypes = [i64, dbl, dbl, dbl, dbl, u64, vp, vp]
        lib.gg_batch_fill.argtypes = [i64, i64, i64, vp, vp, vp, u32, u32, u64, vp, vp, vp]
        lib.gg_draw.argtypes = [u64, u64, u64]
        lib.gg_draw.restype = u64
        _lib = lib
    return _lib


def _alloc(m):
    return (np.empty(m, np.int32), np.empty(m, np.int32), np.empty(m, np.uint32))


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def draw(seed: int, tag: int, k: int) -> int:
    return int(_load().gg_draw(seed, tag, k))


def gnm(n: int, m: int, wlo: int = 1, whi: int = 2**31 - 1, seed: int = 1):
    """GNM: u uniform, v uniform over the other n-1 vertices, w uniform on [wlo, whi]."""
    u, v, w = _alloc(m)
    if _load().gg_gnm(n, m, wlo, whi, seed, _ptr(u), _ptr(v), _ptr(w)) != 0:
        raise ValueError("gnm: bad arguments")
    return u, v, w


def rmat(scale: int, m: int, a=0.57, b=0.19, c=0.19, wlo=1, whi=255, permute=True, seed=2):
    """RMAT (Graph500 default quadrant probabilities), Feistel-permuted vertex ids."""
    u, v, w = _alloc(m)
    if _load().gg_rmat(scale, m, a, b, c, wlo, whi, int(permute), seed,
                       _ptr(u), _ptr(v), _ptr(w)) != 0:
        raise ValueError("rmat: bad arguments")
    return u, v, w


def rmat_permute(scale: int, seed: int, x) -> np.ndarray:
    x = np.ascontiguousarray(x, dtype=np.int64)
    out = np.empty_like(x)
    _load().gg_rmat_permute(scale, seed, _ptr(x), len(x), _ptr(out))
    return out


def _take(h, m):
    if not h:
        raise ValueError("bad generator arguments")
    u, v, w = _alloc(m)
    _load().gg_take(h, _ptr(u), _ptr(v), _ptr(w))
    return u, v, w


def grid(rows: int, cols: int, keep: float = 0.8, wmode: int = 0, wlo: int = 1_000_000,
         whi: int = 1_000_000, seed: int = 3):
    """rows x cols 4-neighbour lattice, each edge kept with probability ``keep``."""
    m = ctypes.c_int64(0)
    h = _load().gg_grid_build(rows, cols, keep, wmode, wlo, whi, seed, ctypes.byref(m))
    return _take(h, m.value)


def rgg2d(n: int, r: float, wscale: float = 1e6, seed: int = 4):
    """2D random geometric graph in the unit square, edge iff distance < r."""
    m = ctypes.c_int64(0)
    h = _load().gg_rgg2d_build(n, r, wscale, seed, ctypes.byref(m))
    return _take(h, m.value)


def rgg3d(n: int, r: float, wlo: int = 1, whi: int = 254, seed: int = 7):
    """3D random geometric graph in the unit cube, edge iff distance < r,
    weights uniform on [wlo, whi]."""
    m = ctypes.c_int64(0)
    h = _load().gg_rgg3d_build(n, r, wlo, whi, seed, ctypes.byref(m))
    return _take(h, m.value)


def rgg3d_radius(n: int, avg_deg: float) -> float:
    """Radius giving expected average degree avg_deg in the unit cube
    (boundary effects ignored): (4/3) pi r^3 (n - 1) = avg_deg."""
    return (3.0 * avg_deg / (4.0 * math.pi * (n - 1))) ** (1.0 / 3.0)


def rhg(n: int, avg_deg: float, wlo: int = 1, whi: int = 254, seed: int = 8):
    """Random hyperbolic graph (threshold model, power-law exponent 3) of
    expected average degree about avg_deg, weights uniform on [wlo, whi]."""
    m = ctypes.c_int64(0)
    h = _load().gg_rhg_build(n, avg_deg, wlo, whi, seed, ctypes.byref(m))
    return _take(h, m.value)


def star_forest(stars: int, leaves: int, copies: int, extra_isolated: int, seed: int):
    """An edge case, not a paper family: ``stars`` disjoint stars of ``leaves``
    leaves each, every hub-leaf edge ``copies`` times with weights in [1, 1000),
    ``extra_isolated`` vertices without edges, ids and edge order shuffled.
    One Borůvka round merges every star, after which no edge is live."""
    rng = np.random.default_rng(seed)
    hubs = np.arange(stars) * (leaves + 1)
    hu = np.repeat(hubs, leaves)
    lv = hu + np.tile(np.arange(1, leaves + 1), stars)
    u = np.tile(hu, copies)
    v = np.tile(lv, copies)
    n = stars * (leaves + 1) + extra_isolated
    perm = rng.permutation(n).astype(np.int32)
    u, v = perm[u], perm[v]
    flip = rng.random(len(u)) < 0.5
    u, v = np.where(flip, v, u), np.where(flip, u, v)
    order = rng.permutation(len(u))
    w = rng.integers(1, 1000, len(u)).astype(np.uint32)
    return u[order].astype(np.int32), v[order].astype(np.int32), w, n


def rgg_radius(n: int, avg_deg: float) -> float:
    """Radius giving expected average degree avg_deg (boundary effects ignored)."""
    return math.sqrt(avg_deg / (math.pi * (n - 1)))


def batch_plan(G, lo=8.0, hi=18.0, dlo=4.0, dhi=64.0, seed=6):
    """Sizes of a batch of GNM graphs: n_g = round(2^U[lo,hi]), d_g ~ U[dlo,dhi],
    m_g = round(n_g d_g / 2).  Returns (n[G], m[G]) int64 arrays."""
    n = np.empty(G, np.int64)
    m = np.empty(G, np.int64)
    if _load().gg_batch_plan(G, lo, hi, dlo, dhi, seed, _ptr(n), _ptr(m)) != 0:
        raise ValueError("batch_plan: bad arguments")
    return n, m


def batch_gnm(G, lo=8.0, hi=18.0, dlo=4.0, dhi=64.0, wlo=1, whi=2**31 - 1, seed=6,
              first=0, count=None):
    """Graphs [first, first+count) of the batch, concatenated: returns
    (u, v, w, edge_off[count+1], vert_off[count+1]) with local vertex ids."""
    nf, mf = batch_plan(G, lo, hi, dlo, dhi, seed)
    count = G - first if count is None else count
    n, m = nf[first:first + count], mf[first:first + count]
    eoff = np.zeros(count + 1, np.int64)
    np.cumsum(m, out=eoff[1:])
    voff = np.zeros(count + 1, np.int64)
    np.cumsum(n, out=voff[1:])
    u, v, w = _alloc(int(eoff[-1]))
    if _load().gg_batch_fill(G, first, count, _ptr(nf), _ptr(mf), _ptr(eoff), wlo, whi, seed,
                             _ptr(u), _ptr(v), _ptr(w)) != 0:
        raise ValueError("batch_gnm: bad arguments")
    return u, v, w, eoff, voff


# --------------------------------------------------------------------------
# Named workloads.  Each returns (u, v, w, n).
# --------------------------------------------------------------------------

def _wl_gnm_small():
    n, m = 1 << 16, 1 << 20
    return (*gnm(n, m, 1, 2**31 - 1, seed=1), n)


def _wl_rmat24():
    return (*rmat(24, 1 << 28, wlo=1, whi=255, seed=2), 1 << 24)


def _wl_grid():
    return (*grid(4096, 4096, 0.8, 0, 1_000_000, 1_000_000, seed=3), 4096 * 4096)


def _wl_grid_u255():
    return (*grid(4096, 4096, 0.8, 1, 1, 255, seed=3), 4096 * 4096)


def _wl_rgg():
    n = 1 << 24
    return (*rgg2d(n, rgg_radius(n, 8.0), 1e6, seed=4), n)


def _wl_rmat22():
    return (*rmat(22, 1 << 28, wlo=1, whi=2**31 - 1, seed=5), 1 << 22)


def _wl_rgg3d():
    n = 1 << 24
    return (*rgg3d(n, rgg3d_radius(n, 16.0), 1, 254, seed=7), n)


def _wl_rhg():
    n = 1 << 24
    return (*rhg(n, 16.0, 1, 254, seed=8), n)


WORKLOADS = {
    "gnm_n2^16_m2^20": _wl_gnm_small,
    "rmat_n2^24_m2^28_w255": _wl_rmat24,
    "grid_4096x4096_keep0.8_w1e6": _wl_grid,
    "grid_4096x4096_keep0.8_w255": _wl_grid_u255,
    "rgg2d_n2^24_deg8": _wl_rgg,
    "rmat_n2^22_m2^28_w2^31": _wl_rmat22,
    "rgg3d_n2^24_deg16_w254": _wl_rgg3d,
    "rhg_n2^24_deg16_g3_w254": _wl_rhg,
}


def workload(name: str):
    return WORKLOADS[name]()
