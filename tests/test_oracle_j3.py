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
import os
import shutil
import subprocess
import tempfile

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


# Plausible mistakes in the j = 3 enumeration, each of which the pins above
# must catch (run on a rebuilt copy of the oracle).
MUTANTS = {
    "no_third_node_adjacency": ("(mark_z[v] == st3 ? 1 : 0)", "0"),
    "no_second_node_edge_to_y": (
        "const int64_t in3 = 1 + (w->mark_s[z] == s ? 1 : 0) + (w->mark_y[z] == st ? 1 : 0);",
        "const int64_t in3 = 1 + (w->mark_s[z] == s ? 1 : 0);"),
    "third_event_may_reinfect_z": ("if (v == s || v == y || v == z) continue;",
                                   "if (v == s || v == y) continue;"),
    "no_third_event_from_z": ("for (int t = 0; t < 3; ++t) {", "for (int t = 0; t < 2; ++t) {"),
}


def _quick_suite3(lib_path):
    import ctypes
    lib = ctypes.CDLL(lib_path)
    vp = ctypes.c_void_p
    lib.oracle_ef3.argtypes = [ctypes.c_int32, vp, vp, vp, ctypes.c_int32, vp, vp, vp,
                               ctypes.c_int32]
    lib.oracle_histogram3.argtypes = [ctypes.c_int32, vp, vp, ctypes.c_int32, vp, vp,
                                      ctypes.c_int64]
    lib.oracle_histogram3.restype = ctypes.c_int64
    for pin in PINS:
        src, dst = efref.pin_graph(pin)
        rp, ci = gen.from_edges(pin["n"], src, dst)
        n = rp.size - 1
        N = np.zeros(n, np.int64)
        D = np.zeros(n, np.int64)
        E = np.zeros(n, np.float64)
        lib.oracle_ef3(n, rp.ctypes.data, ci.ctypes.data, None, n, N.ctypes.data, D.ctypes.data,
                       E.ctypes.data, 1)
        s = pin["node"]
        if (int(N[s]), int(D[s])) != (pin["N"], pin["D"]):
            return False
        if abs(E[s] - efref.eval_pin_expr(pin["expr"])) > 1e-12 * max(1.0, abs(E[s])):
            return False
    for seed in range(2):
        rng = np.random.default_rng(seed)
        n = 8
        pairs = [(a, b) for a, b in itertools.combinations(range(n), 2) if rng.random() < 0.45]
        src, dst = (np.array(x, np.int32) for x in zip(*pairs))
        rp, ci = gen.from_edges(n, src, dst)
        adj = [set(ci[rp[v]:rp[v + 1]].tolist()) for v in range(n)]
        for s in range(n):
            d = np.zeros(256, np.int64)
            c = np.zeros(256, np.int64)
            m = lib.oracle_histogram3(n, rp.ctypes.data, ci.ctypes.data, s, d.ctypes.data,
                                      c.ctypes.data, 256)
            got = {int(a): int(b) for a, b in zip(d[:m], c[:m])}
            if got != brute_histogram3(n, adj, s):
                return False
    return True


def test_unmutated_oracle_passes_quick_suite3():
    oracle._load()
    assert _quick_suite3(oracle.LIB_PATH)


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_mistakes_are_caught3(name):
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    old, new = MUTANTS[name]
    with open(oracle.SRC_PATH) as f:
        src = f.read()
    assert src.count(old) == 1, f"mutation site for {name} not found exactly once"
    src = src.replace(old, new)
    with tempfile.TemporaryDirectory() as td:
        c = os.path.join(td, "m.c")
        so = os.path.join(td, "m.so")
        with open(c, "w") as f:
            f.write(src)
        subprocess.run(["gcc", "-O1", "-std=c11", "-fPIC", "-shared", "-fopenmp", c, "-lm",
                        "-o", so], check=True)
        assert not _quick_suite3(so), f"mutant {name} survived the pins"
