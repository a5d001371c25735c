"""Pure-Python checkers used only by the tests to pin the CPU oracle.

Each routine here computes Expected Force (or one of its integer parts) by a
route different from the oracle's, so that agreement pins the oracle to the
paper rather than to itself:

* ``brute_force``: lists the transmission event sequences literally and takes
  each cluster's degree by counting the edges that cross the cluster boundary
  (Sec. 3.3 and the Fig. 1 caption), then evaluates Eq. 1 as printed,
  -sum p log p.
* ``algorithm1_histograms``: the cluster-centric enumeration of Algorithm 1
  (Phase 1: every pair i<j of neighbours of a centre v; Phase 2: d from the
  three degrees minus 4, minus 2 more for a triangle; credits +1, +1, +2).
* ``closed_form_ND``: N_s and D_s from neighbour-degree sums and triangle
  counts, where the triangle counts come from diag(A^3)/2 computed by numpy.
"""
from __future__ import annotations

import math
from collections import defaultdict

import numpy as np


def adjacency_sets(n, row_ptr, col_idx):
    return [set(int(x) for x in col_idx[row_ptr[i]:row_ptr[i + 1]]) for i in range(n)]


def edges_of(n, row_ptr, col_idx):
    out = []
    for u in range(n):
        for v in col_idx[row_ptr[u]:row_ptr[u + 1]]:
            if u < v:
                out.append((u, int(v)))
    return out


def brute_force(n, row_ptr, col_idx, seeds=None):
    """Returns lists (N, D, EF) by literal enumeration of event sequences."""
    adj = adjacency_sets(n, row_ptr, col_idx)
    edges = edges_of(n, row_ptr, col_idx)
    Ns, Ds, EFs = [], [], []
    for s in (range(n) if seeds is None else seeds):
        degs = []
        for y in adj[s]:                      # event 1: s infects y
            for x in (s, y):                  # event 2: an infected node ...
                for z in adj[x]:              # ... infects a susceptible neighbour
                    if z in (s, y):
                        continue
                    J = {s, y, z}
                    d = sum(1 for (a, b) in edges if (a in J) != (b in J))
                    degs.append(d)
        N = len(degs)
        D = sum(degs)
        if D == 0 or N <= 1:
            ef = 0.0
        else:
            ef = -sum((d / D) * math.log(d / D) for d in degs if d > 0)
        Ns.append(N)
        Ds.append(D)
        EFs.append(ef)
    return Ns, Ds, EFs


def brute_force_bitmask(n, adjmask, s):
    """Same enumeration on a graph given as per-node neighbour bitmasks (n<=8);
    the cluster degree is the number of edges leaving J, counted per member as
    popcount(neighbours outside J)."""
    degs = []
    nb = [[j for j in range(n) if adjmask[i] >> j & 1] for i in range(n)]
    for y in nb[s]:
        for x in (s, y):
            for z in nb[x]:
                if z == s or z == y:
                    continue
                J = (1 << s) | (1 << y) | (1 << z)
                d = sum(bin(adjmask[u] & ~J).count("1") for u in (s, y, z))
                degs.append(d)
    N = len(degs)
    D = sum(degs)
    if D == 0 or N <= 1:
        return N, D, 0.0
    return N, D, -sum((d / D) * math.log(d / D) for d in degs if d > 0)


def algorithm1_histograms(n, row_ptr, col_idx):
    """Per-node histograms {d: count} from Algorithm 1 of the paper."""
    adj = adjacency_sets(n, row_ptr, col_idx)
    deg = [len(a) for a in adj]
    H = [defaultdict(int) for _ in range(n)]
    for v in range(n):                                   # Phase 1
        nb = sorted(adj[v])
        for a in range(len(nb)):
            for b in range(a + 1, len(nb)):
                i, j = nb[a], nb[b]
                d = deg[v] + deg[i] + deg[j] - 4         # Phase 2
                if i in adj[j]:
                    d -= 2
                H[i][d] += 1
                H[j][d] += 1
                H[v][d] += 2
    return [dict(h) for h in H]


def entropy_from_histogram(h):
    N = sum(h.values())
    D = sum(d * c for d, c in h.items())
    if D == 0 or N <= 1:
        return 0.0
    return -sum(c * (d / D) * math.log(d / D) for d, c in h.items() if d > 0)


def dense_adjacency(n, row_ptr, col_idx):
    A = np.zeros((n, n), dtype=np.int64)
    for u in range(n):
        A[u, col_idx[row_ptr[u]:row_ptr[u + 1]]] = 1
    return A


def closed_form_ND(n, row_ptr, col_idx):
    """N_s = k^2 - 2k + A_s and
    D_s = k(k-1)(k-4) + 2(k-1)A + (k-4)(A-k) + (B-A) + (Q-k^2) - 8T_s,
    with A = sum of neighbour degrees, B = sum of their squares, Q = sum over
    neighbours a of (sum of a's neighbour degrees), T_s = triangles at s
    (diag(A^3)/2 of the adjacency matrix)."""
    Adj = dense_adjacency(n, row_ptr, col_idx)
    k = Adj.sum(1)
    A = Adj @ k
    B = Adj @ (k * k)
    sigma = Adj @ k
    Q = Adj @ sigma
    T = np.diag(Adj @ Adj @ Adj) // 2
    N = k * k - 2 * k + A
    D = k * (k - 1) * (k - 4) + 2 * (k - 1) * A + (k - 4) * (A - k) + (B - A) + (Q - k * k) - 8 * T
    return N.astype(np.int64), D.astype(np.int64)


def load_pins(path):
    pins = []
    with open(path) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            parts = [p.strip() for p in line.split("|")]
            name, n, edges, node, N, D, expr, num = parts[:8]
            pins.append(dict(name=name, n=int(n), edges=edges, node=int(node), N=int(N),
                             D=int(D), expr=expr, value=float(num)))
    return pins


def pin_graph(pin):
    """Edge arrays for a pin line."""
    if pin["edges"] == "HUB":
        src = [0] * 1000 + [1001, 1002, 1002]
        dst = list(range(1, 1001)) + [1002, 0, 1003]
    else:
        src, dst = [], []
        for e in pin["edges"].split(","):
            u, v = e.split("-")
            src.append(int(u))
            dst.append(int(v))
    return np.array(src, np.int32), np.array(dst, np.int32)


def eval_pin_expr(expr):
    return float(eval(expr, {"__builtins__": {}}, {"log": math.log}))
