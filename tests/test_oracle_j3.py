"""Pins of the j = 3 oracle (three transmission events, Sec. 3.3).

The oracle enumerates event sequences one by one. It is checked against
  * hand-derived values (tests/golden/ef3_pins.txt);
  * the identity N_3(s) = D_2(s): every two-event sequence with cluster
    degree d extends by exactly d third events (one per edge leaving the
    cluster), so the j = 3 sequence count equals the j = 2 degree sum, which
    the pinned j = 2 oracle gives;
  * a brute force over node orderings on tiny graphs: for every ordered
    triple of new nodes, the number of event sequences infecting them in that
    order is the product, over the three, of their infected neighbours at the
    time; the cluster degree comes from the adjacency matrix.
"""
import itertools
import math

import numpy as np
import pytest

import oracle
from paper_2306_00606_amd import gen
from tests import efref

PINS = efref.load_pins(efref.__file__.replace("efref.py", "golden/ef3_pins.txt"))


@pytest.mark.parametrize("pin", PINS, ids=[p["name"] for p in PINS])
def test_hand_pins(pin):
    src, dst = efref.pin_graph(pin)
    rp, ci = gen.from_edges(pin["n"], src, dst)
    N, D, E = oracle.ef(rp, ci, seeds=[pin["node"]], j=3)
    assert (int(N[0]), int(D[0])) == (pin["N"], pin["D"])
    want = efref.eval_pin_expr(pin["expr"])
    assert abs(E[0] - want) <= 1e-12 * max(1.0, abs(want))
    assert abs(want - pin["value"]) <= 1e-10


def test_closed_forms():
    # K_n: 6 (n-1)(n-2)(n-3) sequences, every cluster degree 4n - 16
    for n in (5, 6, 9):
        src, dst = zip(*itertools.combinations(range(n), 2))
        rp, ci = gen.from_edges(n, np.array(src, np.int32), np.array(dst, np.int32))
        N, D, E = oracle.ef(rp, ci, j=3)
        want_n = 6 * (n - 1) * (n - 2) * (n - 3)
        assert np.all(N == want_n) and np.all(D == want_n * (4 * n - 16))
        assert np.allclose(E, math.log(want_n), rtol=1e-13, atol=0)
    # star with L leaves: centre L(L-1)(L-2), leaf (L-1)(L-2), degree L - 3
    for L in (4, 7):
        rp, ci = gen.from_edges(L + 1, np.zeros(L, np.int32), np.arange(1, L + 1, dtype=np.int32))
        N, D, E = oracle.ef(rp, ci, j=3)
        assert N[0] == L * (L - 1) * (L - 2) and D[0] == N[0] * (L - 3)
        assert np.all(N[1:] == (L - 1) * (L - 2)) and np.all(D[1:] == N[1:] * (L - 3))
        assert np.allclose(E, np.log(N.astype(np.float64)), rtol=1e-13, atol=0)
    # cycles of length >= 5: 8 sequences, degree 2
    for n in (5, 8):
        rp, ci = gen.from_edges(n, np.arange(n, dtype=np.int32),
                                np.roll(np.arange(n, dtype=np.int32), -1))
        N, D, E = oracle.ef(rp, ci, j=3)
        assert np.all(N == 8) and np.all(D == 16) and np.allclose(E, math.log(8), rtol=1e-13)


@pytest.mark.parametrize("graph", ["er200", "rmat9", "ba300", "cm300"])
def test_sequence_count_equals_two_event_degree_sum(graph):
    rp, ci = {
        "er200": lambda: gen.erdos_renyi(200, 8.0 / 199, 4),
        "rmat9": lambda: gen.rmat(9, 8, 3, perm_seed=1),
        "ba300": lambda: gen.barabasi_albert(300, 4, 2),
        "cm300": lambda: gen.config_model(300, 2.3, 5),
    }[graph]()
    N3, D3, E3 = oracle.ef(rp, ci, j=3, threads=4)
    N2, D2, E2 = oracle.ef(rp, ci, j=2, threads=4)
    assert np.array_equal(N3, D2)
    assert np.all(E3 >= 0) and not np.any(np.signbit(E3))


def brute_histogram3(n, adj, s):
    """Histogram of cluster degrees over event sequences, by node orderings."""
    deg = [len(a) for a in adj]
    hist = {}
    others = [v for v in range(n) if v != s]
    for trip in itertools.permutations(others, 3):
        infected = [s]
        ways = 1
        for v in trip:
            ways *= sum(1 for u in infected if u in adj[v])
            infected.append(v)
        if ways == 0:
            continue
        J = [s, *trip]
        inner = sum(1 for a, b in itertools.combinations(J, 2) if b in adj[a])
        d = sum(deg[u] for u in J) - 2 * inner
        hist[d] = hist.get(d, 0) + ways
    return hist


@pytest.mark.parametrize("seed", range(6))
def test_brute_force_node_orderings(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(5, 11))
    p = float(rng.uniform(0.2, 0.7))
    pairs = [(a, b) for a, b in itertools.combinations(range(n), 2) if rng.random() < p]
    if not pairs:
        pairs = [(0, 1)]
    src, dst = (np.array(x, np.int32) for x in zip(*pairs))
    rp, ci = gen.from_edges(n, src, dst)
    adj = [set(ci[rp[v]:rp[v + 1]].tolist()) for v in range(n)]
    for s in range(n):
        assert oracle.histogram(rp, ci, s, j=3) == brute_histogram3(n, adj, s), (seed, s)
