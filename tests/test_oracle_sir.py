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


# --------------------------------------------------------------------------
# The model at fractional beta and mu (Sec. 3.1): statistical pins against
# closed forms, each with planted mistakes that they must catch.
# --------------------------------------------------------------------------
import ctypes  # noqa: E402
import math  # noqa: E402
import os  # noqa: E402
import shutil  # noqa: E402
import subprocess  # noqa: E402
import tempfile  # noqa: E402


def _sir_runner(lib_path=None):
    """oracle.sir, or the same entry point of another build of sir_oracle.c."""
    if lib_path is None:
        return oracle.sir
    lib = ctypes.CDLL(lib_path)
    vp = ctypes.c_void_p
    lib.oracle_sir.argtypes = [ctypes.c_int32, vp, vp, ctypes.c_double, ctypes.c_double,
                               ctypes.c_uint64, ctypes.c_int32, ctypes.c_int32, vp, vp, vp, vp,
                               vp, vp]
    lib.oracle_sir.restype = ctypes.c_int

    def run(rp, ci, beta, mu, seed, n_sims, t_max=100000):
        n = rp.size - 1
        ci = ci if ci.size else np.zeros(1, np.int32)
        o = {k: np.zeros(n_sims, np.int32) for k in ("index", "size", "t_end", "t_peak")}
        o["sp_sum"] = np.zeros((4, n), np.int64)
        o["inf_count"] = np.zeros(n, np.int64)
        st = lib.oracle_sir(n, rp.ctypes.data, ci.ctypes.data, beta, mu, ctypes.c_uint64(seed),
                            n_sims, t_max, o["index"].ctypes.data, o["size"].ctypes.data,
                            o["t_end"].ctypes.data, o["t_peak"].ctypes.data,
                            o["sp_sum"].ctypes.data, o["inf_count"].ctypes.data)
        assert st == 0
        return o
    return run


def _star(k):
    return gen.from_edges(k + 1, np.zeros(k, np.int32), np.arange(1, k + 1, dtype=np.int32))


def _pin_first_generation_binomial(sir):
    """Star with k = 40 leaves, mu = 1: the centre attempts each leaf once,
    so from the centre size - 1 ~ Binomial(40, beta)."""
    k, beta = 40, 0.3
    rp, ci = _star(k)
    o = sir(rp, ci, beta, 1.0, 41, 40000)
    x = o["size"][o["index"] == 0].astype(np.float64) - 1.0
    m = x.size
    if m < 500:
        return False
    mean, var = k * beta, k * beta * (1 - beta)
    # mean within 5 standard errors; the variance within 25% (its standard
    # error is about 5% at this sample size)
    return abs(x.mean() - mean) < 5 * math.sqrt(var / m) and abs(x.var() / var - 1) < 0.25


def _pin_geometric_period(sir):
    """No edges: the index case stays infected for T ~ Geometric(mu) steps
    (P(T = t) = mu (1 - mu)^(t - 1)), and t_end = T."""
    mu, sims = 0.25, 20000
    rp, ci = gen.from_edges(10, [], [])
    o = sir(rp, ci, 0.5, mu, 5, sims)
    t = o["t_end"].astype(np.float64)
    mean, var = 1 / mu, (1 - mu) / mu ** 2
    p1 = float(np.mean(t == 1))
    # memoryless: the share of T = 2 among T >= 2 is mu again
    p2 = float(np.sum(t == 2)) / max(1.0, float(np.sum(t >= 2)))
    se1 = math.sqrt(mu * (1 - mu) / sims)
    return (abs(t.mean() - mean) < 5 * math.sqrt(var / sims) and abs(p1 - mu) < 5 * se1
            and abs(p2 - mu) < 5 * math.sqrt(mu * (1 - mu) / max(1.0, float(np.sum(t >= 2)))))


def _pin_attempts_every_step(sir):
    """Star with k = 40 leaves, beta = 0.1, mu = 0.2, from the centre: the
    centre attempts every still susceptible leaf in each of its T infected
    steps, so a leaf escapes with probability E[(1 - beta)^T] and
    E[size - 1] = k (1 - mu (1 - beta) / (1 - (1 - mu)(1 - beta)))."""
    k, beta, mu = 40, 0.1, 0.2
    rp, ci = _star(k)
    o = sir(rp, ci, beta, mu, 17, 40000)
    x = o["size"][o["index"] == 0].astype(np.float64) - 1.0
    m = x.size
    if m < 500:
        return False
    want = k * (1 - mu * (1 - beta) / (1 - (1 - mu) * (1 - beta)))
    return abs(x.mean() - want) < 5 * x.std() / math.sqrt(m)


SIR_PINS = [_pin_first_generation_binomial, _pin_geometric_period, _pin_attempts_every_step]


@pytest.mark.parametrize("pin", SIR_PINS, ids=[p.__name__[5:] for p in SIR_PINS])
def test_fractional_rates(pin):
    assert pin(_sir_runner())


# Planted mistakes in a copy of sir_oracle.c: (site, replacement) pairs.
SIR_MUTANTS = {
    # a node attempts only in the first step it is infected
    "attempt_first_step_only": [
        ("memset(state, S_SUS, (size_t)n);",
         "memset(state, S_SUS, (size_t)n); memset(was_inf, 0, (size_t)n);"),
        ("if (state[u] != S_INF) continue;\n        for (int32_t e = row_ptr[u];",
         "if (state[u] != S_INF || was_inf[u]) continue;\n        was_inf[u] = 1;\n"
         "        for (int32_t e = row_ptr[u];"),
    ],
    # recovery ignores mu: every infected node recovers after one step
    "always_recover": [("if ((x >> 11) < tm) state[u] = S_REC;\n        else ++next;",
                        "state[u] = S_REC;\n        (void)x;")],
    # attempts drawn with the recovery probability
    "beta_mu_swapped": [("if ((x >> 11) < tb && u < cand[w])", "if ((x >> 11) < tm && u < cand[w])")],
    # recovery decided before the attempts of the step (recovered nodes do not attempt)
    "recover_before_attempt": [
        ("if (state[u] != S_INF) continue;\n        for (int32_t e = row_ptr[u];",
         "if (state[u] != S_INF) continue;\n"
         "        if ((mix(st ^ ((uint64_t)(2 * (int64_t)u + 1) * 0xD1B54A32D192ED03ull)) >> 11) < tm)"
         " continue;\n        for (int32_t e = row_ptr[u];"),
    ],
}


@pytest.mark.parametrize("name", sorted(SIR_MUTANTS))
def test_sir_planted_mistakes_are_caught(name):
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    with open(oracle.SIR_SRC_PATH) as f:
        src = f.read()
    for old, new in SIR_MUTANTS[name]:
        assert src.count(old) == 1, f"mutation site for {name} not found exactly once: {old!r}"
        src = src.replace(old, new)
    with tempfile.TemporaryDirectory() as td:
        c = os.path.join(td, "m.c")
        so = os.path.join(td, "m.so")
        with open(c, "w") as f:
            f.write(src)
        subprocess.run(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", c, "-o", so], check=True)
        run = _sir_runner(so)
        caught = [p.__name__ for p in SIR_PINS if not p(run)]
    assert caught, f"mutant {name} survived every fractional-rate pin"
