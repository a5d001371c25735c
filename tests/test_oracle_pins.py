"""Pins of the CPU oracle to the paper and to mathematics (no GPU).

The oracle (``oracle/ef_oracle.c``) is checked against: hand-derived values
(``tests/golden/ef_pins.txt``), literal brute force over every labelled graph
on up to 6 nodes, the cluster-centric enumeration of Algorithm 1, closed
forms for the integer parts, and invariants (sum rules, entropy bounds,
relabelling, disjoint union). ``test_planted_mistakes_are_caught`` plants
plausible mistakes in a copy of the oracle and checks that these pins catch
each one.
"""
from __future__ import annotations

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

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "ef_pins.txt")
PINS = efref.load_pins(GOLDEN)


def _close(a, b, rel=1e-12, abs_=1e-15):
    return abs(a - b) <= max(abs_, rel * abs(b))


@pytest.mark.parametrize("pin", PINS, ids=[p["name"] for p in PINS])
def test_golden_pin(pin):
    src, dst = efref.pin_graph(pin)
    rp, ci = gen.from_edges(pin["n"], src, dst)
    N, D, E = oracle.ef(rp, ci, seeds=[pin["node"]])
    assert int(N[0]) == pin["N"] and int(D[0]) == pin["D"]
    expect = efref.eval_pin_expr(pin["expr"])
    assert _close(expect, pin["value"], rel=1e-10, abs_=1e-12)
    assert _close(float(E[0]), expect), (float(E[0]), expect)
    assert math.copysign(1.0, float(E[0])) > 0  # never -0.0


@pytest.mark.parametrize("pin", PINS, ids=[p["name"] for p in PINS])
def test_golden_pin_matches_brute_force(pin):
    src, dst = efref.pin_graph(pin)
    rp, ci = gen.from_edges(pin["n"], src, dst)
    N, D, E = efref.brute_force(pin["n"], rp, ci, seeds=[pin["node"]])
    assert (N[0], D[0]) == (pin["N"], pin["D"])
    assert _close(E[0], efref.eval_pin_expr(pin["expr"]), rel=1e-11)


def _all_graphs(n):
    pairs = list(itertools.combinations(range(n), 2))
    for mask in range(1 << len(pairs)):
        yield [pairs[i] for i in range(len(pairs)) if mask >> i & 1]


@pytest.mark.parametrize("n", [3, 4, 5, 6])
def test_exhaustive_small_graphs_vs_brute_force(n):
    """Every labelled simple graph on n nodes, all seeds, in one disjoint union."""
    graphs = list(_all_graphs(n))
    src, dst = [], []
    for g, edges in enumerate(graphs):
        for (u, v) in edges:
            src.append(g * n + u)
            dst.append(g * n + v)
    total = len(graphs) * n
    rp, ci = gen.from_edges(total, np.array(src, np.int32), np.array(dst, np.int32))
    N, D, E = oracle.ef(rp, ci)
    for g, edges in enumerate(graphs):
        adjmask = [0] * n
        for (u, v) in edges:
            adjmask[u] |= 1 << v
            adjmask[v] |= 1 << u
        for s in range(n):
            bn, bd, be = efref.brute_force_bitmask(n, adjmask, s)
            t = g * n + s
            assert (int(N[t]), int(D[t])) == (bn, bd), (edges, s)
            assert _close(float(E[t]), be, rel=1e-12, abs_=1e-14), (edges, s, E[t], be)


def _random_graphs():
    yield "er30", gen.erdos_renyi(30, 0.2, 7)
    yield "er40", gen.erdos_renyi(40, 0.25, 11)
    yield "ba80", gen.barabasi_albert(80, 3, 5)
    yield "rmat7", gen.rmat(7, 6, 3, perm_seed=9)
    yield "ws60", gen.watts_strogatz(60, 6, 0.2, 4)
    yield "cm80", gen.config_model(80, 2.2, 6)


@pytest.mark.parametrize("name,g", list(_random_graphs()))
def test_random_graphs_vs_brute_force(name, g):
    rp, ci = g
    n = rp.size - 1
    N, D, E = oracle.ef(rp, ci)
    bN, bD, bE = efref.brute_force(n, rp, ci)
    assert list(N) == bN and list(D) == bD
    for a, b in zip(E, bE):
        assert _close(float(a), b, rel=1e-11, abs_=1e-14)


@pytest.mark.parametrize("name,g", list(_random_graphs()))
def test_histograms_equal_algorithm1(name, g):
    """The oracle's per-seed histograms equal the per-node histograms that
    Algorithm 1 builds cluster-centrically (multiplicities +2/+1/+1, -2 for
    triangles)."""
    rp, ci = g
    n = rp.size - 1
    H = efref.algorithm1_histograms(n, rp, ci)
    for s in range(n):
        assert oracle.histogram(rp, ci, s) == H[s], s
    N, D, E = oracle.ef(rp, ci)
    for s in range(n):
        assert _close(float(E[s]), efref.entropy_from_histogram(H[s]), rel=1e-11, abs_=1e-14)


@pytest.mark.parametrize("name,g", list(_random_graphs()) + [
    ("ba400", gen.barabasi_albert(400, 4, 2)), ("rmat9", gen.rmat(9, 8, 1, perm_seed=2))])
def test_closed_form_integers(name, g):
    rp, ci = g
    n = rp.size - 1
    N, D, _ = oracle.ef(rp, ci)
    cN, cD = efref.closed_form_ND(n, rp, ci)
    assert np.array_equal(N, cN)
    assert np.array_equal(D, cD)


def test_sum_rules_and_entropy_bounds():
    rp, ci = gen.rmat(11, 8, 5, perm_seed=6)
    n = rp.size - 1
    deg = np.diff(rp).astype(np.int64)
    W = int((deg * (deg - 1) // 2).sum())
    N, D, E = oracle.ef(rp, ci)
    assert int(N.sum()) == 4 * W                       # every cluster counted 4 times
    # sum of D = 4 * sum over Algorithm 1's clusters of their degree
    src = np.repeat(np.arange(n), deg)
    lo = src < ci
    T = 0
    adj = efref.adjacency_sets(n, rp, ci)
    sumd = 0
    for v in range(n):
        nb = np.sort(ci[rp[v]:rp[v + 1]])
        kv = deg[v]
        kn = deg[nb]
        tot = (kv - 4) * len(nb) * (len(nb) - 1) // 2 + (len(nb) - 1) * int(kn.sum())
        tri = sum(1 for a, b in itertools.combinations(nb.tolist(), 2) if b in adj[a])
        sumd += tot - 2 * tri
        T += tri
    assert int(D.sum()) == 4 * sumd
    assert lo.sum() * 2 == rp[-1]
    ok = N > 0
    assert np.all(E >= 0.0)
    assert np.all(E[ok] <= np.log(N[ok]) + 1e-12)
    assert np.all(E[N <= 1] == 0.0)


def test_entropy_upper_bound_attained_when_degrees_equal():
    # cycles and cliques: every cluster of a seed has the same degree
    for n in (5, 9):
        rp, ci = gen.from_edges(n, np.arange(n), (np.arange(n) + 1) % n)
        N, D, E = oracle.ef(rp, ci)
        assert np.allclose(E, np.log(N), rtol=0, atol=1e-14)
    rp, ci = gen.erdos_renyi(7, 1.0, 0)
    N, D, E = oracle.ef(rp, ci)
    assert np.allclose(E, np.log(N), rtol=0, atol=1e-14)


def test_relabel_invariance():
    rp, ci = gen.barabasi_albert(500, 4, 12)
    n = rp.size - 1
    N, D, E = oracle.ef(rp, ci)
    perm = np.random.default_rng(0).permutation(n).astype(np.int32)
    deg = np.diff(rp)
    src = np.repeat(np.arange(n, dtype=np.int32), deg)
    rp2, ci2 = gen.from_edges(n, perm[src], perm[ci])
    N2, D2, E2 = oracle.ef(rp2, ci2)
    assert np.array_equal(N2[perm], N) and np.array_equal(D2[perm], D)
    assert np.array_equal(E2[perm], E)


def test_disjoint_union_and_isolated_node():
    g1 = gen.erdos_renyi(60, 0.1, 1)
    g2 = gen.barabasi_albert(50, 2, 3)
    parts = []
    off = 0
    for rp, ci in (g1, g2):
        n = rp.size - 1
        src = np.repeat(np.arange(n, dtype=np.int32), np.diff(rp)) + off
        parts.append((src, ci + off))
        off += n
    src = np.concatenate([p[0] for p in parts])
    dst = np.concatenate([p[1] for p in parts])
    rpu, ciu = gen.from_edges(off + 1, src, dst)   # one extra isolated node at the end
    Nu, Du, Eu = oracle.ef(rpu, ciu)
    N1, D1, E1 = oracle.ef(*g1)
    N2, D2, E2 = oracle.ef(*g2)
    assert np.array_equal(Nu[:-1], np.concatenate([N1, N2]))
    assert np.array_equal(Du[:-1], np.concatenate([D1, D2]))
    assert np.array_equal(Eu[:-1], np.concatenate([E1, E2]))
    assert (Nu[-1], Du[-1], Eu[-1]) == (0, 0, 0.0)


def test_thread_count_does_not_change_results():
    rp, ci = gen.barabasi_albert(3000, 5, 8)
    a = oracle.ef(rp, ci, threads=1)
    b = oracle.ef(rp, ci, threads=4)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


def test_selected_seeds_position_aligned():
    rp, ci = gen.erdos_renyi(200, 0.05, 3)
    N, D, E = oracle.ef(rp, ci)
    seeds = np.array([5, 5, 0, 199, 17], np.int32)
    Ns, Ds, Es = oracle.ef(rp, ci, seeds=seeds)
    assert np.array_equal(Ns, N[seeds]) and np.array_equal(Ds, D[seeds])
    assert np.array_equal(Es, E[seeds])


# --------------------------------------------------------------------------
# Planted mistakes: each mutant of the oracle source must fail a pin.
# --------------------------------------------------------------------------

MUTANTS = {
    "drop_star_triangle_test": (
        "const int64_t internal = 1 /* s~y */ + 1 /* s~z */ + (w->mark_y[z] == st ? 1 : 0);",
        "const int64_t internal = 1 /* s~y */ + 1 /* s~z */;"),
    "drop_path_triangle_test": (
        "const int64_t internal = 1 /* s~y */ + 1 /* y~z */ + (w->mark_s[z] == s ? 1 : 0);",
        "const int64_t internal = 1 /* s~y */ + 1 /* y~z */;"),
    "star_counted_once": (
        "if (z == y || z == s) continue;",
        "if (z <= y || z == s) continue;"),
    "drop_path_events": (
        "for (int32_t e2 = y0; e2 < y1; ++e2) {",
        "for (int32_t e2 = y0; e2 < y0; ++e2) {"),
    "wrong_sign_internal": (
        "hist_add(w, ks + ky + kz - 2 * internal);\n    }\n    /* event 2 by y",
        "hist_add(w, ks + ky + kz - 1 * internal);\n    }\n    /* event 2 by y"),
    "entropy_transposed": (
        "log1p((double)(D - d) / (double)d)",
        "log1p((double)(D - d) / Dd)"),
    "count_entropy_not_degree_weighted": (
        "(double)w->hist[d] * ((double)d / Dd) * log1p((double)(D - d) / (double)d);",
        "(double)w->hist[d] / (double)N * log((double)N / (double)w->hist[d]);"),
    "path_z_may_equal_s": (
        "if (z == s || z == y) continue;",
        "if (z == y) continue;"),
}


def _quick_pin_suite(lib_path):
    """A fast subset of the pins, run against a given oracle build."""
    import ctypes
    lib = ctypes.CDLL(lib_path)
    vp = ctypes.c_void_p
    lib.oracle_ef.argtypes = [ctypes.c_int32, vp, vp, vp, ctypes.c_int32, vp, vp, vp,
                              ctypes.c_int32]

    def run(rp, ci):
        n = rp.size - 1
        N = np.zeros(n, np.int64)
        D = np.zeros(n, np.int64)
        E = np.zeros(n, np.float64)
        lib.oracle_ef(n, rp.ctypes.data, ci.ctypes.data, None, n, N.ctypes.data,
                      D.ctypes.data, E.ctypes.data, 1)
        return N, D, E

    for pin in PINS:
        src, dst = efref.pin_graph(pin)
        rp, ci = gen.from_edges(pin["n"], src, dst)
        N, D, E = run(rp, ci)
        s = pin["node"]
        if (int(N[s]), int(D[s])) != (pin["N"], pin["D"]):
            return False
        if not _close(float(E[s]), efref.eval_pin_expr(pin["expr"])):
            return False
    for _, (rp, ci) in list(_random_graphs())[:2]:
        n = rp.size - 1
        N, D, E = run(rp, ci)
        bN, bD, bE = efref.brute_force(n, rp, ci)
        if list(N) != bN or list(D) != bD:
            return False
        if not all(_close(float(a), b, rel=1e-11, abs_=1e-14) for a, b in zip(E, bE)):
            return False
    return True


def test_unmutated_oracle_passes_quick_suite():
    oracle._load()
    assert _quick_pin_suite(oracle.LIB_PATH)


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_mistakes_are_caught(name):
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
        assert not _quick_pin_suite(so), f"mutant {name} survived the pins"


# --------------------------------------------------------------------------
# The surrogate MLP oracle: hand-written gradients pinned by finite differences
# --------------------------------------------------------------------------

def test_mlp_oracle_gradients_match_finite_differences():
    from oracle import mlp_ref
    rs = np.random.default_rng(3)
    p = mlp_ref.init_params(1)
    p["b1"] = rs.normal(0, 0.1, 64)
    p["b2"] = rs.normal(0, 0.1, 64)
    p["b3"] = np.array([0.3])
    X = rs.normal(0, 1, (7, 16))
    t = rs.normal(0, 1, 7)
    loss, g = mlp_ref.loss_and_grads(p, X, t)
    h = 1e-6
    for name in ("W1", "b1", "W2", "b2", "w3", "b3"):
        flat = p[name].reshape(-1)
        for idx in rs.choice(flat.size, min(6, flat.size), replace=False):
            old = flat[idx]
            flat[idx] = old + h
            lp, _ = mlp_ref.loss_and_grads(p, X, t)
            flat[idx] = old - h
            lm, _ = mlp_ref.loss_and_grads(p, X, t)
            flat[idx] = old
            fd = (lp - lm) / (2 * h)
            an = g[name].reshape(-1)[idx]
            assert abs(fd - an) <= 1e-6 * max(1.0, abs(fd)), (name, idx, fd, an)


def test_mlp_oracle_gelu_and_bf16_rounding():
    from oracle import mlp_ref
    import math
    # gelu(0) = 0, gelu(x) -> x for large x, gelu(-x) -> 0; derivative at 0 is 1/2
    assert mlp_ref.gelu(np.array([0.0]))[0] == 0.0
    assert abs(mlp_ref.gelu(np.array([10.0]))[0] - 10.0) < 1e-12
    assert abs(mlp_ref.gelu(np.array([-10.0]))[0]) < 1e-12
    assert abs(mlp_ref.gelu_grad(np.array([0.0]))[0] - 0.5) < 1e-15
    # the tanh form stays within 1e-3 of the erf form (its published accuracy)
    z = np.linspace(-6, 6, 241)
    exact = 0.5 * z * (1 + np.vectorize(math.erf)(z / math.sqrt(2)))
    assert np.max(np.abs(mlp_ref.gelu(z) - exact)) < 1e-3
    # bfloat16 keeps 8 significant bits, ties to even
    assert mlp_ref.bf16_round(np.array([1.0]))[0] == 1.0
    assert mlp_ref.bf16_round(np.array([1.0 + 2 ** -8]))[0] == 1.0          # tie -> even
    assert mlp_ref.bf16_round(np.array([1.0 + 3 * 2 ** -8]))[0] == 1.0 + 2 ** -6
    assert mlp_ref.bf16_round(np.array([-3.0]))[0] == -3.0


def test_spearman_reference():
    from oracle import mlp_ref
    from scipy.stats import spearmanr
    rs = np.random.default_rng(0)
    a = rs.integers(0, 20, 300).astype(float)   # with ties
    b = a + rs.normal(0, 3, 300)
    assert abs(mlp_ref.spearman(a, b) - spearmanr(a, b).correlation) < 1e-12
