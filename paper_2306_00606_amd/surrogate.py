"""Training loop and evaluation of the learned EF surrogate.

Labelled sets come from the exact kernel of this library (cluster-centric,
FP32C) on graphs drawn from the three exact-path generators at training
scale: Erdős–Rényi (n 1e3..1e5, mean degree 4..16), Barabási–Albert
(n 1e4..1e6, m 2..10) and R-MAT (scale 12..18, edge factor 4..16). Targets are
y = ln N(s) - EF(s); features are the library's 16 per-node features.
Training, prediction and rescoring all run on the GPU through efgpu.
"""
from __future__ import annotations

import math
import time

import numpy as np

from . import efgpu, gen


def training_graphs(seed: int = 0, count: int = 18, small: bool = False):
    """Graphs of the three generator families; `small` shrinks them for tests."""
    rs = np.random.default_rng(seed)
    out = []
    for i in range(count):
        fam = i % 3
        s = int(rs.integers(1, 2 ** 31))
        if fam == 0:
            n = int(rs.integers(1000, 5000 if small else 100_000))
            k = float(rs.uniform(4, 16))
            out.append(("er", gen.erdos_renyi(n, k / (n - 1), s)))
        elif fam == 1:
            n = int(rs.integers(2000 if small else 10_000, 20_000 if small else 1_000_000))
            m = int(rs.integers(2, 11))
            out.append(("ba", gen.barabasi_albert(n, m, s)))
        else:
            scale = int(rs.integers(10 if small else 12, 13 if small else 19))
            ef = int(rs.integers(4, 17))
            out.append(("rmat", gen.rmat(scale, ef, s, perm_seed=s + 1)))
    return out


def labelled_rows(graphs, prec: str = "fp32c"):
    """Features X (rows x 16) and targets y = ln N - EF from the exact kernel."""
    Xs, ys = [], []
    for _, (rp, ci) in graphs:
        with efgpu.Graph(rp, ci, validate=False) as g:
            ef, _, _ = g.compute(algo="cluster", prec=prec)
            X, lnN = g.features()
        Xs.append(X)
        ys.append((lnN.astype(np.float64) - ef).astype(np.float32))
    return np.concatenate(Xs), np.concatenate(ys)


def top_overlap(score, exact, frac: float = 0.01):
    """|top(score) & top(exact)| / m with m = ceil(frac n), ties by node id."""
    n = len(exact)
    m = max(1, int(math.ceil(frac * n)))
    ids = np.arange(n)
    a = np.lexsort((ids, -np.asarray(score, np.float64)))[:m]
    b = np.lexsort((ids, -np.asarray(exact, np.float64)))[:m]
    return len(np.intersect1d(a, b)) / m


def spearman(a, b):
    from scipy.stats import spearmanr
    return float(spearmanr(a, b).correlation)


def _median_event_ms(fn, reps: int = 10) -> float:
    """Median over `reps` calls of fn, each timed with HIP events on the
    current stream (the library's calls run on it), after one warm-up call."""
    import torch

    fn()
    times = []
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        fn()
        b.record()
        b.synchronize()
        times.append(a.elapsed_time(b))
    return float(np.median(times))


def evaluate(sur: efgpu.Surrogate, graph: efgpu.Graph, exact=None):
    """Spearman and top-1% overlap of the surrogate and of the non-learned
    proxies ln N(s) and degree, against exact EF; and the time of each (median
    of 10 event-timed calls, device outputs)."""
    import torch

    dev = torch.device("cuda:0")
    ef_d = torch.empty(graph.n, dtype=torch.float64, device=dev)
    D_d = torch.empty(graph.n, dtype=torch.int64, device=dev)
    N_d = torch.empty(graph.n, dtype=torch.int64, device=dev)
    t_exact = 1e-3 * _median_event_ms(
        lambda: graph.compute(algo="cluster", prec="fp32c", out=(ef_d, D_d, N_d)))
    if exact is None:
        exact = ef_d.cpu().numpy()
    # prediction (features + MLP), device output
    out = torch.empty(graph.n, dtype=torch.float64, device="cuda:0")
    t_pred = 1e-3 * _median_event_ms(lambda: sur.predict(graph, out=out))
    pred = out.cpu().numpy()
    X, lnN = graph.features()
    deg = np.expm1(X[:, 0].astype(np.float64))
    res = {
        "n": graph.n,
        "surrogate": {"spearman": spearman(pred, exact), "top1pct": top_overlap(pred, exact)},
        "ln_N": {"spearman": spearman(lnN, exact), "top1pct": top_overlap(lnN, exact)},
        "degree": {"spearman": spearman(deg, exact), "top1pct": top_overlap(deg, exact)},
        "t_exact_ms": 1e3 * t_exact,
        "t_surrogate_ms": 1e3 * t_pred,
    }
    res["speedup"] = t_exact / t_pred if t_pred > 0 else None
    return res
