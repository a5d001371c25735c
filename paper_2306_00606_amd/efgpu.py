"""Python binding of ``libef.so`` (the C-ABI declared in ``include/ef.h``).

Argument marshalling only: every step of the computation runs in the
library's HIP kernels. PyTorch, when given, only supplies device memory and
the current HIP stream. There is no CPU fallback: if the library is missing or
no gfx950 device is visible, calls raise.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libef.so")

# status codes (ef_status)
EF_OK = 0
STATUS_NAMES = {
    0: "EF_OK", 1: "EF_ERR_ARG", 2: "EF_ERR_NOT_SYMMETRIC", 3: "EF_ERR_SELF_LOOP",
    4: "EF_ERR_DUPLICATE", 5: "EF_ERR_UNSORTED", 6: "EF_ERR_RANGE", 7: "EF_ERR_OVERFLOW",
    8: "EF_ERR_NOMEM", 9: "EF_ERR_DEVICE", 10: "EF_ERR_STATE",
}
ALGO = {"cluster": 0, "per_seed": 1, "cluster_agg": 2}
PREC = {"fp64": 0, "fp32c": 1}
EF_VALIDATE = 0x1
EF_DEVICE_PTRS = 0x2
EF_OUT_DEVICE = 0x4
EF_PROFILE = 0x8
EF_BATCH_PHASED = 0x10
EF_BATCH_PERSISTENT = 0x20

# every entry point declared in include/ef.h
EXPORTS = [
    "ef_last_error", "ef_version", "ef_device_count", "ef_validate_csr", "ef_graph_load_csr",
    "ef_graph_from_edges", "ef_graph_free", "ef_graph_info_get", "ef_compute", "ef_compute_j3",
    "ef_topk", "ef_topk_values", "ef_topk_values_noalloc",
    "ef_stats", "ef_batch_create", "ef_batch_autotune", "ef_batch_compute",
    "ef_batch_stats_get", "ef_batch_free", "ef_surrogate_create", "ef_surrogate_free",
    "ef_surrogate_get_params", "ef_surrogate_set_params", "ef_surrogate_save",
    "ef_surrogate_load", "ef_features", "ef_surrogate_gradients", "ef_surrogate_forward",
    "ef_surrogate_train",
    "ef_surrogate_predict", "ef_topk_surrogate", "ef_sir",
]

N_FEATURES = 16
N_PARAMS = 5313


class EFError(RuntimeError):
    def __init__(self, status: int, message: str):
        self.status = status
        self.name = STATUS_NAMES.get(status, str(status))
        super().__init__(f"{self.name}: {message}")


class GraphInfo(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("nnz", ctypes.c_int64), ("max_degree", ctypes.c_int32),
                ("clusters", ctypes.c_int64), ("sum_sq_degree", ctypes.c_int64),
                ("up_arcs", ctypes.c_int64), ("wedge_checks", ctypes.c_int64)]


class RunStats(ctypes.Structure):
    _fields_ = [("t_bin_ms", ctypes.c_double), ("t_pairs_ms", ctypes.c_double),
                ("t_pairs_small_ms", ctypes.c_double), ("t_pairs_mid_ms", ctypes.c_double),
                ("t_pairs_big_ms", ctypes.c_double), ("t_reduce_ms", ctypes.c_double),
                ("t_triangles_ms", ctypes.c_double), ("t_stream_ms", ctypes.c_double),
                ("t_finalize_ms", ctypes.c_double), ("t_pass2_ms", ctypes.c_double),
                ("t_total_ms", ctypes.c_double), ("pairs_small", ctypes.c_int64),
                ("pairs_mid", ctypes.c_int64), ("pairs_big", ctypes.c_int64),
                ("pair_tiles", ctypes.c_int64), ("promoted", ctypes.c_int64),
                ("fp64_finalized", ctypes.c_int64), ("seeds", ctypes.c_int64)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class BatchStats(ctypes.Structure):
    _fields_ = [("n_graphs", ctypes.c_int32), ("n", ctypes.c_int32), ("nnz", ctypes.c_int64),
                ("clusters", ctypes.c_int64), ("replay_ms", ctypes.c_double),
                ("tune_ms", ctypes.c_float * 8), ("tuned_choice", ctypes.c_int32),
                ("thr8", ctypes.c_int32), ("thr16", ctypes.c_int32), ("thr32", ctypes.c_int32),
                ("persist_tune_ms", ctypes.c_float * 8), ("persist_choice", ctypes.c_int32),
                ("design", ctypes.c_int32), ("items", ctypes.c_int32),
                ("from_cache", ctypes.c_int32), ("size_class", ctypes.c_int32),
                ("persist_pass2", ctypes.c_int32), ("persist_fp64", ctypes.c_int32)]

    def as_dict(self):
        d = {f: getattr(self, f) for f, _ in self._fields_}
        d["tune_ms"] = list(self.tune_ms)
        d["persist_tune_ms"] = list(self.persist_tune_ms)
        return d


class TrainCfg(ctypes.Structure):
    _fields_ = [("lr", ctypes.c_float), ("epochs", ctypes.c_int32), ("batch", ctypes.c_int32),
                ("seed", ctypes.c_uint64), ("weight_decay", ctypes.c_float),
                ("val_fraction", ctypes.c_float), ("patience", ctypes.c_int32),
                ("lr_end", ctypes.c_float)]


class TrainReport(ctypes.Structure):
    _fields_ = [("epochs_run", ctypes.c_int32), ("train_loss", ctypes.c_float),
                ("val_loss", ctypes.c_float), ("train_ms", ctypes.c_float),
                ("rows", ctypes.c_int64), ("val_rows", ctypes.c_int64)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class JudgeReport(ctypes.Structure):
    _fields_ = [("candidates", ctypes.c_int32), ("sample", ctypes.c_int32),
                ("spearman", ctypes.c_float), ("fallback", ctypes.c_int32),
                ("t_predict_ms", ctypes.c_float), ("t_rescore_ms", ctypes.c_float),
                ("t_judge_ms", ctypes.c_float)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


_lib = None


def _preload_hip_runtime():
    """Load PyTorch's HIP runtime (by path, globally) before libef.so, so that
    torch and this library share one runtime in the process: the same device
    allocations and the same stream objects."""
    import importlib.util

    spec = importlib.util.find_spec("torch")
    if spec and spec.submodule_search_locations:
        rt = os.path.join(spec.submodule_search_locations[0], "lib", "libamdhip64.so")
        if os.path.exists(rt):
            ctypes.CDLL(rt, mode=ctypes.RTLD_GLOBAL)


def lib():
    """Load libef.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                           "(there is no CPU fallback)")
    _preload_hip_runtime()
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, u32 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32
    L.ef_last_error.restype = ctypes.c_char_p
    L.ef_last_error.argtypes = []
    L.ef_version.restype = i32
    L.ef_device_count.argtypes = [ctypes.POINTER(i32)]
    L.ef_validate_csr.argtypes = [i32, i64, vp, vp]
    L.ef_graph_load_csr.argtypes = [i32, i64, vp, vp, u32, vp, ctypes.POINTER(vp)]
    L.ef_graph_from_edges.argtypes = [i32, i64, vp, vp, vp, ctypes.POINTER(vp)]
    L.ef_graph_free.argtypes = [vp]
    L.ef_graph_info_get.argtypes = [vp, ctypes.POINTER(GraphInfo)]
    L.ef_compute.argtypes = [vp, ctypes.c_int, ctypes.c_int, vp, i32, vp, vp, vp, u32, vp]
    L.ef_compute_j3.argtypes = [vp, ctypes.c_int, vp, i32, vp, vp, vp, u32, vp]
    L.ef_sir.argtypes = [vp, ctypes.c_double, ctypes.c_double, ctypes.c_uint64, i32, i32, vp, vp,
                         vp, vp, vp, vp, vp, vp, vp]
    L.ef_stats.argtypes = [vp, ctypes.POINTER(RunStats)]
    L.ef_topk.argtypes = [vp, ctypes.c_int, ctypes.c_int, i32, vp, vp, u32, vp]
    L.ef_topk_values.argtypes = [vp, vp, i32, vp, vp, u32, vp]
    L.ef_topk_values_noalloc.argtypes = [vp, i32, i32, vp, vp, u32, vp]
    L.ef_batch_create.argtypes = [i32, vp, i64, vp, vp, u32, vp, ctypes.POINTER(vp)]
    L.ef_batch_autotune.argtypes = [vp, ctypes.c_int]
    L.ef_batch_compute.argtypes = [vp, ctypes.c_int, vp, vp, vp, u32, vp]
    L.ef_batch_stats_get.argtypes = [vp, ctypes.POINTER(BatchStats)]
    L.ef_batch_free.argtypes = [vp]
    L.ef_surrogate_create.argtypes = [ctypes.c_uint64, ctypes.POINTER(vp)]
    L.ef_surrogate_free.argtypes = [vp]
    L.ef_surrogate_get_params.argtypes = [vp, vp, vp, vp]
    L.ef_surrogate_set_params.argtypes = [vp, vp, vp, vp]
    L.ef_surrogate_save.argtypes = [vp, ctypes.c_char_p]
    L.ef_surrogate_load.argtypes = [vp, ctypes.c_char_p]
    L.ef_features.argtypes = [vp, vp, vp, u32, vp]
    L.ef_surrogate_gradients.argtypes = [vp, vp, vp, i64, vp, vp, vp]
    L.ef_surrogate_forward.argtypes = [vp, vp, i64, vp, u32, vp]
    L.ef_surrogate_train.argtypes = [vp, vp, vp, i64, ctypes.POINTER(TrainCfg),
                                     ctypes.POINTER(TrainReport), vp]
    L.ef_surrogate_predict.argtypes = [vp, vp, vp, u32, vp]
    L.ef_topk_surrogate.argtypes = [vp, vp, i32, i32, i32, ctypes.c_float, ctypes.c_uint64, vp,
                                    vp, ctypes.POINTER(JudgeReport), vp]
    for name in EXPORTS[2:]:
        getattr(L, name).restype = ctypes.c_int
    _lib = L
    return L


def last_error() -> str:
    return lib().ef_last_error().decode()


def _check(status: int):
    if status != EF_OK:
        raise EFError(status, last_error())


def topk_values_noalloc(ef, k: int, nodes, values=None, stream=None):
    """ef_topk_values_noalloc: top-k of the device tensor `ef` (float64) into
    the caller's device tensors `nodes` (int32, >= k) and `values` (float64 or
    None), without any allocation; asynchronous on the stream."""
    _check(lib().ef_topk_values_noalloc(ef.data_ptr(), int(ef.numel()), int(k), nodes.data_ptr(),
                                        values.data_ptr() if values is not None else None,
                                        EF_OUT_DEVICE, _stream_ptr(stream)))
    return nodes, values


def device_count() -> int:
    c = ctypes.c_int32(0)
    _check(lib().ef_device_count(ctypes.byref(c)))
    return int(c.value)


def validate_csr(row_ptr, col_idx):
    rp = np.ascontiguousarray(row_ptr, dtype=np.int32)
    ci = np.ascontiguousarray(col_idx, dtype=np.int32)
    n = rp.size - 1
    _check(lib().ef_validate_csr(n, int(ci.size), rp.ctypes.data,
                                 ci.ctypes.data if ci.size else None))


def _is_torch(x):
    return type(x).__module__.startswith("torch")


def _stream_ptr(stream):
    if stream is not None:
        return ctypes.c_void_p(int(stream))
    try:
        import torch
        if torch.cuda.is_available():
            return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    except Exception:
        pass
    return None


class Graph:
    """A graph loaded into device memory (opaque handle ``ef_graph``)."""

    def __init__(self, row_ptr, col_idx, validate: bool = True, stream=None):
        self._h = ctypes.c_void_p()
        flags = EF_VALIDATE if validate else 0
        if _is_torch(row_ptr) and row_ptr.is_cuda:
            # borrowed device arrays: keep references alive
            self._keep = (row_ptr.contiguous(), col_idx.contiguous())
            rp, ci = self._keep
            assert rp.dtype == ci.dtype and str(rp.dtype) == "torch.int32"
            n, nnz = rp.numel() - 1, ci.numel()
            flags |= EF_DEVICE_PTRS
            _check(lib().ef_graph_load_csr(n, nnz, rp.data_ptr(), ci.data_ptr() if nnz else None,
                                           flags, _stream_ptr(stream), ctypes.byref(self._h)))
        else:
            rp = np.ascontiguousarray(row_ptr, dtype=np.int32)
            ci = np.ascontiguousarray(col_idx, dtype=np.int32)
            n, nnz = rp.size - 1, ci.size
            _check(lib().ef_graph_load_csr(n, nnz, rp.ctypes.data,
                                           ci.ctypes.data if nnz else None, flags,
                                           _stream_ptr(stream), ctypes.byref(self._h)))
        self.n = n
        self.nnz = nnz

    @classmethod
    def from_edges(cls, n, src, dst, stream=None):
        self = cls.__new__(cls)
        self._h = ctypes.c_void_p()
        s = np.ascontiguousarray(src, dtype=np.int32)
        d = np.ascontiguousarray(dst, dtype=np.int32)
        _check(lib().ef_graph_from_edges(int(n), int(s.size), s.ctypes.data, d.ctypes.data,
                                         _stream_ptr(stream), ctypes.byref(self._h)))
        self.n = int(n)
        self.nnz = self.info()["nnz"]
        return self

    def info(self) -> dict:
        inf = GraphInfo()
        _check(lib().ef_graph_info_get(self._h, ctypes.byref(inf)))
        return {f: getattr(inf, f) for f, _ in GraphInfo._fields_}

    def stats(self) -> dict:
        st = RunStats()
        _check(lib().ef_stats(self._h, ctypes.byref(st)))
        return st.as_dict()

    def compute(self, algo: str = "cluster", prec: str = "fp32c", seeds=None,
                out=None, profile: bool = False, stream=None, j: int = 2):
        """EF (and exact D, N) of all nodes or of `seeds`, for j = 2 (the
        paper's setting; `algo` picks the formulation) or j = 3 transmission
        events (ef_compute_j3; `algo` is not used).

        Host mode (out=None): returns numpy (ef float64, D int64, N int64).
        Device mode: `out` = (ef, D, N) torch CUDA tensors (D, N may be None);
        the call is asynchronous on `stream` (default: torch's current stream).
        """
        if j not in (2, 3):
            raise ValueError("j must be 2 or 3")
        flags = EF_PROFILE if profile else 0

        def call(p_ef, p_D, p_N, fl):
            if j == 3:
                return lib().ef_compute_j3(self._h, PREC[prec], sp, ns, p_ef, p_D, p_N, fl,
                                           _stream_ptr(stream))
            return lib().ef_compute(self._h, ALGO[algo], PREC[prec], sp, ns, p_ef, p_D, p_N, fl,
                                    _stream_ptr(stream))
        if seeds is not None:
            sd = np.ascontiguousarray(seeds, dtype=np.int32)
            ns = sd.size
            sp = sd.ctypes.data if ns else None
        else:
            sd, ns, sp = None, 0, None
        count = ns if seeds is not None else self.n
        if out is None:
            ef = np.zeros(max(count, 1), np.float64)
            D = np.zeros(max(count, 1), np.int64)
            N = np.zeros(max(count, 1), np.int64)
            _check(call(ef.ctypes.data, D.ctypes.data, N.ctypes.data, flags))
            return ef[:count], D[:count], N[:count]
        ef, D, N = out
        _check(call(ef.data_ptr(), D.data_ptr() if D is not None else None,
                    N.data_ptr() if N is not None else None, flags | EF_OUT_DEVICE))
        return ef, D, N

    def topk(self, k: int, algo: str = "cluster", prec: str = "fp32c", out=None,
             profile: bool = False, stream=None):
        """The k nodes of largest EF (descending; ties by id ascending).
        Host mode returns numpy (nodes int32, ef float64); device mode writes
        `out` = (nodes, ef) torch CUDA tensors asynchronously."""
        flags = EF_PROFILE if profile else 0
        if out is None:
            nodes = np.zeros(max(k, 1), np.int32)
            ef = np.zeros(max(k, 1), np.float64)
            _check(lib().ef_topk(self._h, ALGO[algo], PREC[prec], int(k), nodes.ctypes.data,
                                 ef.ctypes.data, flags, _stream_ptr(stream)))
            return nodes[:k], ef[:k]
        nodes, ef = out
        _check(lib().ef_topk(self._h, ALGO[algo], PREC[prec], int(k), nodes.data_ptr(),
                             ef.data_ptr() if ef is not None else None, flags | EF_OUT_DEVICE,
                             _stream_ptr(stream)))
        return nodes, ef

    def topk_values(self, ef, k: int, out=None, stream=None):
        """Top-k selection over EF values already on the device (`ef`: a torch
        CUDA float64 tensor of n values). Host mode returns numpy (nodes, ef);
        device mode writes `out` = (nodes, ef) torch CUDA tensors."""
        if out is None:
            nodes = np.zeros(max(k, 1), np.int32)
            val = np.zeros(max(k, 1), np.float64)
            _check(lib().ef_topk_values(self._h, ef.data_ptr(), int(k), nodes.ctypes.data,
                                        val.ctypes.data, 0, _stream_ptr(stream)))
            return nodes[:k], val[:k]
        nodes, val = out
        _check(lib().ef_topk_values(self._h, ef.data_ptr(), int(k), nodes.data_ptr(),
                                    val.data_ptr() if val is not None else None, EF_OUT_DEVICE,
                                    _stream_ptr(stream)))
        return nodes, val

    def sir(self, beta: float, mu: float, seed: int, n_sims: int, t_max: int = 100000,
            profile: bool = False, stream=None) -> dict:
        """SIR outbreaks (ef_sir): per-simulation index, size, t_end, t_peak and,
        over the global outbreaks, inf_count[v] and sp_sum[d-1, v] (d = 1..4);
        work = (arcs walked by the attempts, frontier node-steps); with profile,
        phase_ms = kernel time of attempts, updates and descendant counts."""
        n = self.n
        out = {"index": np.zeros(max(n_sims, 1), np.int32),
               "size": np.zeros(max(n_sims, 1), np.int32),
               "t_end": np.zeros(max(n_sims, 1), np.int32),
               "t_peak": np.zeros(max(n_sims, 1), np.int32),
               "sp_sum": np.zeros((4, max(n, 1)), np.int64),
               "inf_count": np.zeros(max(n, 1), np.int64),
               "work": np.zeros(2, np.int64)}
        ph = np.zeros(3, np.float64)
        _check(lib().ef_sir(self._h, float(beta), float(mu), ctypes.c_uint64(seed & (2**64 - 1)),
                            int(n_sims), int(t_max), out["index"].ctypes.data,
                            out["size"].ctypes.data, out["t_end"].ctypes.data,
                            out["t_peak"].ctypes.data, out["sp_sum"].ctypes.data,
                            out["inf_count"].ctypes.data, out["work"].ctypes.data,
                            ph.ctypes.data if profile else None, _stream_ptr(stream)))
        for k in ("index", "size", "t_end", "t_peak"):
            out[k] = out[k][:n_sims]
        out["sp_sum"] = out["sp_sum"][:, :n]
        out["inf_count"] = out["inf_count"][:n]
        if profile:
            out["phase_ms"] = {"attempts": ph[0], "updates": ph[1], "descendants": ph[2]}
        return out

    def features(self):
        """Raw per-node features (n x 16, float32) and ln N (float32)."""
        X = np.zeros((max(self.n, 1), N_FEATURES), np.float32)
        L = np.zeros(max(self.n, 1), np.float32)
        _check(lib().ef_features(self._h, X.ctypes.data, L.ctypes.data, 0, _stream_ptr(None)))
        return X[:self.n], L[:self.n]

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            lib().ef_graph_free(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


def union_csr(graphs):
    """Disjoint union of [(row_ptr, col_idx), ...]: (node_off, row_ptr, col_idx)."""
    node_off = np.zeros(len(graphs) + 1, np.int64)
    for i, (rp, _) in enumerate(graphs):
        node_off[i + 1] = node_off[i] + (len(rp) - 1)
    nnz = sum(int(rp[-1]) for rp, _ in graphs)
    rp_u = np.zeros(int(node_off[-1]) + 1, np.int64)
    ci_u = np.zeros(nnz, np.int32)
    arc = 0
    for i, (rp, ci) in enumerate(graphs):
        n0, n1 = int(node_off[i]), int(node_off[i + 1])
        rp_u[n0 + 1:n1 + 1] = arc + rp[1:].astype(np.int64)
        ci_u[arc:arc + ci.size] = ci + n0
        arc += ci.size
    return node_off.astype(np.int32), rp_u.astype(np.int32), ci_u


class Batch:
    """Many graphs computed together (handle ``ef_batch``): one disjoint union,
    computed by the phased or the persistent design, each captured once as a
    HIP graph and replayed per call."""

    def __init__(self, graphs, validate: bool = False, stream=None):
        node_off, rp, ci = union_csr(graphs)
        self.node_off = node_off
        self.n = int(node_off[-1])
        self._h = ctypes.c_void_p()
        _check(lib().ef_batch_create(len(graphs), node_off.ctypes.data, int(ci.size),
                                     rp.ctypes.data, ci.ctypes.data if ci.size else None,
                                     EF_VALIDATE if validate else 0, _stream_ptr(stream),
                                     ctypes.byref(self._h)))

    def autotune(self, prec: str = "fp32c"):
        _check(lib().ef_batch_autotune(self._h, PREC[prec]))

    def compute(self, prec: str = "fp32c", out=None, profile: bool = False, stream=None,
                design: str | None = None):
        """design: None (the tuned one), "phased" or "persistent"."""
        flags = (EF_PROFILE if profile else 0) | {None: 0, "phased": EF_BATCH_PHASED,
                                                  "persistent": EF_BATCH_PERSISTENT}[design]
        if out is None:
            ef = np.zeros(max(self.n, 1), np.float64)
            D = np.zeros(max(self.n, 1), np.int64)
            N = np.zeros(max(self.n, 1), np.int64)
            _check(lib().ef_batch_compute(self._h, PREC[prec], ef.ctypes.data, D.ctypes.data,
                                          N.ctypes.data, flags, _stream_ptr(stream)))
            return ef[:self.n], D[:self.n], N[:self.n]
        ef, D, N = out
        _check(lib().ef_batch_compute(self._h, PREC[prec], ef.data_ptr(),
                                      D.data_ptr() if D is not None else None,
                                      N.data_ptr() if N is not None else None,
                                      flags | EF_OUT_DEVICE, _stream_ptr(stream)))
        return ef, D, N

    def split(self, arr):
        """Per-graph views of a per-node array of the union."""
        return [arr[self.node_off[i]:self.node_off[i + 1]] for i in range(len(self.node_off) - 1)]

    def stats(self) -> dict:
        st = BatchStats()
        _check(lib().ef_batch_stats_get(self._h, ctypes.byref(st)))
        return st.as_dict()

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            lib().ef_batch_free(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


class Surrogate:
    """The learned EF surrogate (handle ``ef_surrogate``)."""

    def __init__(self, seed: int = 0):
        self._h = ctypes.c_void_p()
        _check(lib().ef_surrogate_create(int(seed), ctypes.byref(self._h)))

    def params(self):
        P = np.zeros(N_PARAMS, np.float32)
        m = np.zeros(N_FEATURES, np.float32)
        s = np.zeros(N_FEATURES, np.float32)
        _check(lib().ef_surrogate_get_params(self._h, P.ctypes.data, m.ctypes.data, s.ctypes.data))
        return P, m, s

    def set_params(self, P=None, mean=None, inv_std=None):
        arrs = [None if a is None else np.ascontiguousarray(a, np.float32) for a in (P, mean, inv_std)]
        _check(lib().ef_surrogate_set_params(self._h, *[None if a is None else a.ctypes.data
                                                         for a in arrs]))

    def save(self, path):
        _check(lib().ef_surrogate_save(self._h, str(path).encode()))

    def load(self, path):
        _check(lib().ef_surrogate_load(self._h, str(path).encode()))

    def gradients(self, X, y):
        X = np.ascontiguousarray(X, np.float32)
        y = np.ascontiguousarray(y, np.float32)
        g = np.zeros(N_PARAMS, np.float32)
        loss = ctypes.c_float()
        _check(lib().ef_surrogate_gradients(self._h, X.ctypes.data, y.ctypes.data, len(y),
                                            g.ctypes.data, ctypes.byref(loss), _stream_ptr(None)))
        return g, float(loss.value)

    def forward(self, X):
        """The network's output for rows of 16 (standardised) inputs."""
        X = np.ascontiguousarray(X, np.float32)
        y = np.zeros(max(X.shape[0], 1), np.float32)
        _check(lib().ef_surrogate_forward(self._h, X.ctypes.data, X.shape[0], y.ctypes.data, 0,
                                          _stream_ptr(None)))
        return y[:X.shape[0]]

    def train(self, X, y, lr=3e-3, epochs=30, batch=4096, seed=0, weight_decay=0.0,
              val_fraction=0.05, patience=4, lr_end=0.05):
        X = np.ascontiguousarray(X, np.float32)
        y = np.ascontiguousarray(y, np.float32)
        cfg = TrainCfg(lr, epochs, batch, seed, weight_decay, val_fraction, patience, lr_end)
        rep = TrainReport()
        _check(lib().ef_surrogate_train(self._h, X.ctypes.data, y.ctypes.data, len(y),
                                        ctypes.byref(cfg), ctypes.byref(rep), _stream_ptr(None)))
        return rep.as_dict()

    def predict(self, graph: Graph, out=None, stream=None):
        if out is None:
            ef = np.zeros(max(graph.n, 1), np.float64)
            _check(lib().ef_surrogate_predict(self._h, graph._h, ef.ctypes.data, 0,
                                              _stream_ptr(stream)))
            return ef[:graph.n]
        _check(lib().ef_surrogate_predict(self._h, graph._h, out.data_ptr(), EF_OUT_DEVICE,
                                          _stream_ptr(stream)))
        return out

    def topk(self, graph: Graph, k: int, rerank_factor: int = 4, judge_sample: int = 4096,
             min_spearman: float = 0.98, seed: int = 0):
        nodes = np.zeros(max(k, 1), np.int32)
        ef = np.zeros(max(k, 1), np.float64)
        rep = JudgeReport()
        _check(lib().ef_topk_surrogate(graph._h, self._h, int(k), int(rerank_factor),
                                       int(judge_sample), float(min_spearman), int(seed),
                                       nodes.ctypes.data, ef.ctypes.data, ctypes.byref(rep),
                                       _stream_ptr(None)))
        return nodes[:k], ef[:k], rep.as_dict()

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            lib().ef_surrogate_free(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
