"""Pins of the SIR oracle (Sec. 3.1 model, Sec. 3.3 spreading power).

* SplitMix64, the counter-based generator behind every random decision,
  against its published first output for state 0.
* With beta = 1 and mu = 1 the outbreak is deterministic: every infected
  node infects all susceptible neighbours and recovers in the same step, so
  the outbreak is a breadth-first search from the index case, each node's
  infector being its smallest-id neighbour one layer closer. Sizes, durations,
  peaks and the depth-limited descendant sums are checked against an
  independent breadth-first search written here.
* With beta = 0 nothing spreads; with mu = 1 the index case recovers after
  one step.
* The index cases are uniform over the nodes (chi-square on many draws).
"""
import collections

import numpy as np
import pytest

import oracle
from paper_2306_00606_amd import gen


def test_splitmix64_published_value():
    assert oracle.splitmix64(0) == 0xE220A8397B1DCDAF


def bfs_outbreak(rp, ci, idx):
    n = rp.size - 1
    dist = {idx: 0}
    parent = {idx: -1}
    layer = [idx]
    while layer:
        nxt = []
        for u in sorted(layer):
            for w in ci[rp[u]:rp[u + 1]]:
                w = int(w)
                if w not in dist:
                    dist[w] = dist[u] + 1
                    parent[w] = u  # sorted layer: the smallest infector first
                    nxt.append(w)
        layer = nxt
    children = collections.defaultdict(list)
    for v, p in parent.items():
        if p >= 0:
            children[p].append(v)

    def desc(v, d):
        if d == 0:
            return 0
        return sum(1 + desc(c, d - 1) for c in children[v])

    ecc = max(dist.values())
    layers = collections.Counter(dist.values())
    peak_t = max(layers, key=lambda t: (layers[t], -t))
    sp = {v: [desc(v, d) for d in range(1, 5)] for v in dist}
    return len(dist), ecc + 1, peak_t, sp


@pytest.mark.parametrize("graph", ["er60", "ws50", "tree"])
def test_deterministic_outbreak_is_bfs(graph):
    rp, ci = {
        "er60": lambda: gen.erdos_renyi(60, 0.06, 3),
        "ws50": lambda: gen.watts_strogatz(50, 4, 0.2, 1),
        "tree": lambda: gen.from_edges(15, np.arange(1, 15, dtype=np.int32),
                                       (np.arange(1, 15) - 1) // 2),
    }[graph]()
    n = rp.size - 1
    o = oracle.sir(rp, ci, 1.0, 1.0, seed=11, n_sims=12)
    want_sp = np.zeros((4, n), np.int64)
    want_cnt = np.zeros(n, np.int64)
    for r in range(12):
        size, t_end, t_peak, sp = bfs_outbreak(rp, ci, int(o["index"][r]))
        assert (o["size"][r], o["t_end"][r], o["t_peak"][r]) == (size, t_end, t_peak), r
        if size >= (n + 3) // 4:
            for v, s in sp.items():
                want_sp[:, v] += s
                want_cnt[v] += 1
    assert np.array_equal(o["sp_sum"], want_sp)
    assert np.array_equal(o["inf_count"], want_cnt)


def test_no_spread_and_immediate_recovery():
    rp, ci = gen.er_1000(2)
    o = oracle.sir(rp, ci, 0.0, 1.0, seed=5, n_sims=50)
    assert np.all(o["size"] == 1) and np.all(o["t_end"] == 1) and np.all(o["t_peak"] == 0)
    assert o["inf_count"].sum() == 0  # no global outbreak


def test_index_cases_are_uniform():
    rp, ci = gen.from_edges(10, np.arange(9, dtype=np.int32), np.arange(1, 10, dtype=np.int32))
    o = oracle.sir(rp, ci, 0.0, 1.0, seed=3, n_sims=20000)
    counts = np.bincount(o["index"], minlength=10)
    chi2 = float(((counts - 2000.0) ** 2 / 2000.0).sum())
    assert chi2 < 27.9  # 9 degrees of freedom, p = 0.001
