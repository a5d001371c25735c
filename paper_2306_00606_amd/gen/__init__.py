"""Seeded synthetic graph generators (ctypes over ``libefgen.so``).

Input plumbing only: no Expected Force arithmetic lives here. The CPU
oracle's tests, the GPU library's tests and the benchmark all draw their
graphs from this module, so the two sides see identical inputs.

Every function returns ``(row_ptr, col_idx)`` as int32 numpy arrays describing
a simple undirected graph (both arc directions stored, rows sorted, no
self-loops or duplicates; isolated nodes kept).
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libefgen.so")


class _Csr(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int32),
        ("nnz", ctypes.c_int64),
        ("row_ptr", ctypes.POINTER(ctypes.c_int32)),
        ("col_idx", ctypes.POINTER(ctypes.c_int32)),
    ]


_lib = None


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        from .. import build as _build

        _build.build_gen()
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.POINTER(_Csr)
    lib.efgen_free.argtypes = [P]
    lib.efgen_free.restype = None
    lib.efgen_from_edges.argtypes = [ctypes.c_int32, ctypes.c_int64,
                                     ctypes.c_void_p, ctypes.c_void_p]
    lib.efgen_from_edges.restype = P
    lib.efgen_er.argtypes = [ctypes.c_int32, ctypes.c_double, ctypes.c_uint64]
    lib.efgen_er.restype = P
    lib.efgen_ba.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_uint64]
    lib.efgen_ba.restype = P
    lib.efgen_rmat.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_double,
                               ctypes.c_double, ctypes.c_double, ctypes.c_uint64,
                               ctypes.c_uint64]
    lib.efgen_rmat.restype = P
    lib.efgen_ws.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_double,
                             ctypes.c_uint64]
    lib.efgen_ws.restype = P
    lib.efgen_cm.argtypes = [ctypes.c_int32, ctypes.c_double, ctypes.c_int32,
                             ctypes.c_uint64]
    lib.efgen_cm.restype = P
    _lib = lib
    return lib


def _take(p):
    if not p:
        raise ValueError("generator rejected its arguments")
    c = p.contents
    n, nnz = int(c.n), int(c.nnz)
    rp = np.ctypeslib.as_array(c.row_ptr, shape=(n + 1,)).copy()
    ci = (np.ctypeslib.as_array(c.col_idx, shape=(nnz,)).copy()
          if nnz else np.zeros(0, np.int32))
    _load().efgen_free(p)
    return rp.astype(np.int32, copy=False), ci.astype(np.int32, copy=False)


def from_edges(n: int, src, dst):
    src = np.ascontiguousarray(src, dtype=np.int32)
    dst = np.ascontiguousarray(dst, dtype=np.int32)
    assert src.shape == dst.shape
    return _take(_load().efgen_from_edges(int(n), int(src.size),
                                          src.ctypes.data, dst.ctypes.data))


def erdos_renyi(n: int, p: float, seed: int):
    return _take(_load().efgen_er(int(n), float(p), int(seed)))


def barabasi_albert(n: int, m: int, seed: int):
    return _take(_load().efgen_ba(int(n), int(m), int(seed)))


def rmat(scale: int, edge_factor: int, seed: int, a: float = 0.57, b: float = 0.19,
         c: float = 0.19, perm_seed: int = 0):
    return _take(_load().efgen_rmat(int(scale), int(edge_factor), float(a), float(b),
                                    float(c), int(seed), int(perm_seed)))


def watts_strogatz(n: int, k: int, p: float, seed: int):
    return _take(_load().efgen_ws(int(n), int(k), float(p), int(seed)))


def config_model(n: int, gamma: float, seed: int, kmin: int = 2):
    return _take(_load().efgen_cm(int(n), float(gamma), int(kmin), int(seed)))


# ---------------------------------------------------------------------------
# The named workloads. Each recipe is fixed here so that tests and benchmark
# build identical graphs.
# ---------------------------------------------------------------------------

@dataclass(frozen=True)
class Workload:
    name: str
    description: str


def er_1000(seed: int = 1):
    """Erdos-Renyi G(n=1000, p=8/999): mean degree 8, isolated nodes kept."""
    return erdos_renyi(1000, 8.0 / 999.0, seed)


def ba_1m(seed: int = 2, n: int = 1_000_000, m: int = 5):
    """Barabasi-Albert n=1e6, m=5 (about 5M undirected edges)."""
    return barabasi_albert(n, m, seed)


def rmat_22(seed: int = 1, scale: int = 22, edge_factor: int = 10, perm_seed: int = 3):
    """R-MAT scale 22, edge factor 10, a=.57 b=.19 c=.19 d=.05, symmetrised,
    deduplicated, ids shuffled by a seeded permutation (about 40M edges)."""
    return rmat(scale, edge_factor, seed, 0.57, 0.19, 0.19, perm_seed)


def batch_512(seed0: int = 1000, count: int = 512, n_lo: int = 1000, n_hi: int = 100_000):
    """The mixed batch: half Watts-Strogatz (n ~ U[n_lo, n_hi], k in {4,6,8,10},
    p ~ U[0.01, 0.3]), half erased configuration model (n ~ U[n_lo, n_hi],
    gamma ~ U[2.1, 3.0]). Parameters of graph i come from a generator seeded
    with seed0 + i. Returns a list of (row_ptr, col_idx)."""
    out = []
    for i in range(count):
        rs = np.random.default_rng(seed0 + i)
        n = int(rs.integers(n_lo, n_hi + 1))
        if i % 2 == 0:
            k = int(rs.choice([4, 6, 8, 10]))
            p = float(rs.uniform(0.01, 0.3))
            out.append(watts_strogatz(n, k, p, seed0 + i))
        else:
            g = float(rs.uniform(2.1, 3.0))
            out.append(config_model(n, g, seed0 + i))
    return out
