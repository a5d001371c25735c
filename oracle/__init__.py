"""CPU oracle for Expected Force (ctypes over ``liboracle.so``, built from
``ef_oracle.c``).

TEST INFRASTRUCTURE ONLY. It may be imported by ``tests/``, by
``__graft_entry__.smoke()`` and by the CPU-baseline leg of ``bench.py``;
nothing in the GPU library imports, links or calls it, and it shares no code
with that library.

What it computes is the plain definition: per seed, every ordered pair of
transmission events, the degree of the resulting three-node cluster (edges
leaving it), the histogram of those degrees and the entropy of Eq. 1 of
"Scaling Expected Force" (Sec. 3.3), in double precision, with the
multiplicities of Algorithm 1; and the same with three events (four-node
clusters, the parameter j = 3 of Sec. 3.3). See ``ef_oracle.c`` for the exact
statement. ``sir_oracle.c`` simulates the SIR model of Sec. 3.1 and sums the
empirical spreading power of Sec. 3.3.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")
SRC_PATH = os.path.join(_HERE, "ef_oracle.c")

_lib = None


SIR_SRC_PATH = os.path.join(_HERE, "sir_oracle.c")


def build():
    tmp = LIB_PATH + ".tmp"
    subprocess.run(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", SRC_PATH,
                    SIR_SRC_PATH, "-lm", "-o", tmp], check=True)
    os.replace(tmp, LIB_PATH)


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        build()
    lib = ctypes.CDLL(LIB_PATH)
    vp = ctypes.c_void_p
    lib.oracle_ef.argtypes = [ctypes.c_int32, vp, vp, vp, ctypes.c_int32, vp, vp, vp,
                              ctypes.c_int32]
    lib.oracle_ef.restype = ctypes.c_int
    lib.oracle_histogram.argtypes = [ctypes.c_int32, vp, vp, ctypes.c_int32, vp, vp,
                                     ctypes.c_int64]
    lib.oracle_histogram.restype = ctypes.c_int64
    lib.oracle_ef3.argtypes = lib.oracle_ef.argtypes
    lib.oracle_ef3.restype = ctypes.c_int
    lib.oracle_histogram3.argtypes = lib.oracle_histogram.argtypes
    lib.oracle_histogram3.restype = ctypes.c_int64
    lib.oracle_splitmix64.argtypes = [ctypes.c_uint64]
    lib.oracle_splitmix64.restype = ctypes.c_uint64
    lib.oracle_sir.argtypes = [ctypes.c_int32, vp, vp, ctypes.c_double, ctypes.c_double,
                               ctypes.c_uint64, ctypes.c_int32, ctypes.c_int32, vp, vp, vp, vp,
                               vp, vp]
    lib.oracle_sir.restype = ctypes.c_int
    _lib = lib
    return lib


def _csr(row_ptr, col_idx):
    rp = np.ascontiguousarray(row_ptr, dtype=np.int32)
    ci = np.ascontiguousarray(col_idx, dtype=np.int32)
    if ci.size == 0:
        ci = np.zeros(1, np.int32)
    return rp, ci


def ef(row_ptr, col_idx, seeds=None, threads: int = 1, j: int = 2):
    """Returns (N, D, EF) as int64, int64, float64 arrays aligned with `seeds`
    (all nodes when seeds is None), for j = 2 or j = 3 transmission events."""
    if j not in (2, 3):
        raise ValueError("j must be 2 or 3")
    rp, ci = _csr(row_ptr, col_idx)
    n = rp.size - 1
    if seeds is None:
        cnt = n
        sp = None
    else:
        sd = np.ascontiguousarray(seeds, dtype=np.int32)
        cnt = sd.size
        sp = sd.ctypes.data if cnt else None
    N = np.zeros(max(cnt, 1), np.int64)
    D = np.zeros(max(cnt, 1), np.int64)
    E = np.zeros(max(cnt, 1), np.float64)
    if cnt:
        fn = _load().oracle_ef if j == 2 else _load().oracle_ef3
        st = fn(n, rp.ctypes.data, ci.ctypes.data, sp, cnt, N.ctypes.data, D.ctypes.data,
                E.ctypes.data, int(threads))
        if st != 0:
            raise RuntimeError(f"oracle_ef failed with status {st}")
    return N[:cnt], D[:cnt], E[:cnt]


def histogram(row_ptr, col_idx, s: int, j: int = 2):
    """H_s as a dict {cluster degree: number of event sequences} (j = 2 or 3)."""
    if j not in (2, 3):
        raise ValueError("j must be 2 or 3")
    rp, ci = _csr(row_ptr, col_idx)
    n = rp.size - 1
    lib = _load()
    fn = lib.oracle_histogram if j == 2 else lib.oracle_histogram3
    cap = 64
    while True:
        d = np.zeros(cap, np.int64)
        c = np.zeros(cap, np.int64)
        m = fn(n, rp.ctypes.data, ci.ctypes.data, int(s), d.ctypes.data, c.ctypes.data, cap)
        if m < 0:
            raise RuntimeError("oracle_histogram failed")
        if m <= cap:
            return {int(a): int(b) for a, b in zip(d[:m], c[:m])}
        cap = int(m)


def splitmix64(z: int) -> int:
    """SplitMix64's output function of a 64-bit counter (the oracle's copy)."""
    return int(_load().oracle_splitmix64(ctypes.c_uint64(z & (2**64 - 1))))


def sir(row_ptr, col_idx, beta: float, mu: float, seed: int, n_sims: int, t_max: int = 100000):
    """SIR simulations (Sec. 3.1) and the spreading-power sums over the global
    ones (Sec. 3.3); see sir_oracle.c. Returns a dict of numpy arrays."""
    rp, ci = _csr(row_ptr, col_idx)
    n = rp.size - 1
    out = {"index": np.zeros(max(n_sims, 1), np.int32), "size": np.zeros(max(n_sims, 1), np.int32),
           "t_end": np.zeros(max(n_sims, 1), np.int32),
           "t_peak": np.zeros(max(n_sims, 1), np.int32),
           "sp_sum": np.zeros((4, max(n, 1)), np.int64),
           "inf_count": np.zeros(max(n, 1), np.int64)}
    st = _load().oracle_sir(n, rp.ctypes.data, ci.ctypes.data, float(beta), float(mu),
                            ctypes.c_uint64(seed & (2**64 - 1)), int(n_sims), int(t_max),
                            out["index"].ctypes.data, out["size"].ctypes.data,
                            out["t_end"].ctypes.data, out["t_peak"].ctypes.data,
                            out["sp_sum"].ctypes.data, out["inf_count"].ctypes.data)
    if st != 0:
        raise RuntimeError(f"oracle_sir failed with status {st}")
    for k in ("index", "size", "t_end", "t_peak"):
        out[k] = out[k][:n_sims]
    out["sp_sum"] = out["sp_sum"][:, :n]
    out["inf_count"] = out["inf_count"][:n]
    return out
