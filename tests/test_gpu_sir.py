"""Parity of the GPU SIR simulations (ef_sir) with the CPU oracle (needs an
MI355X). Every output is an integer function of the same counter-based draws,
so the comparison is exact: index cases, sizes, durations, peaks, and the
spreading-power sums and infection counts over the global outbreaks."""
import sys

import numpy as np
import pytest

import oracle
from paper_2306_00606_amd import efgpu, gen

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _announce(request):
    sys.stderr.write(f"\n[gpu case] {request.node.nodeid}\n")
    sys.stderr.flush()
    yield


def paper_beta(rp):
    n = rp.size - 1
    return 1.3 / (3.0 * (rp[-1] / n))


def compare(a, b, what):
    for k in ("index", "size", "t_end", "t_peak", "sp_sum", "inf_count"):
        assert np.array_equal(a[k], b[k]), f"{what}: {k} differs"


CASES = {
    "er1000_paper": (lambda: gen.er_1000(4), None, 1 / 3, 300),
    "er1000_strong": (lambda: gen.er_1000(4), 0.12, 1 / 3, 200),
    "ws2000_strong": (lambda: gen.watts_strogatz(2000, 8, 0.2, 5), 0.2, 1 / 3, 100),
    "ba3000_paper": (lambda: gen.barabasi_albert(3000, 4, 2), None, 1 / 3, 300),
    "cm2000_strong": (lambda: gen.config_model(2000, 2.3, 3), 0.3, 0.5, 100),
    "er500_bfs": (lambda: gen.erdos_renyi(500, 0.01, 9), 1.0, 1.0, 50),
}


@pytest.mark.parametrize("name", sorted(CASES))
def test_sir_matches_oracle(name):
    mk, beta, mu, sims = CASES[name]
    rp, ci = mk()
    beta = paper_beta(rp) if beta is None else beta
    with efgpu.Graph(rp, ci) as g:
        got = g.sir(beta, mu, seed=2024, n_sims=sims)
    want = oracle.sir(rp, ci, beta, mu, seed=2024, n_sims=sims)
    compare(got, want, name)
    n = rp.size - 1
    glob = got["size"] >= (n + 3) // 4
    sys.stderr.write(f"[sir] {name}: {int(glob.sum())} global of {sims}\n")
    assert np.all(got["size"] >= 1) and np.all(got["t_peak"] <= got["t_end"])
    # every infected node but the index case has an infector: order-1 sums
    # over a global outbreak add up to its size - 1
    assert got["sp_sum"][0].sum() == int((got["size"][glob] - 1).sum())
    # work counters: every infected node is in the frontier for at least one
    # step, and each step walks all of its arcs
    assert got["work"][1] >= got["size"].sum() and got["work"][0] >= 0


def test_sir_ba_1m_paper_calibration():
    """BA n = 10^6, m = 5 at the paper's calibration, 100 outbreaks: the size
    the benchmark runs, every output against the oracle."""
    rp, ci = gen.ba_1m(seed=8)
    beta = paper_beta(rp)
    with efgpu.Graph(rp, ci, validate=False) as g:
        got = g.sir(beta, 1 / 3, seed=77, n_sims=100)
    want = oracle.sir(rp, ci, beta, 1 / 3, seed=77, n_sims=100)
    compare(got, want, "BA 1e6, 100 simulations")
    n = rp.size - 1
    glob = got["size"] >= (n + 3) // 4
    sys.stderr.write(f"[sir] BA 1e6: {int(glob.sum())} global of 100\n")
    assert glob.sum() > 0
    assert np.all(got["sp_sum"][1:] >= got["sp_sum"][:-1])  # deeper subtrees are larger


def test_sir_work_counts_bfs():
    """beta = mu = 1: each infected node is in the frontier for exactly one
    step, so the frontier node-steps are the outbreak sizes and the arcs walked
    are the degrees of the infected nodes."""
    rp, ci = gen.config_model(3000, 2.4, 5)
    deg = np.diff(rp)
    with efgpu.Graph(rp, ci) as g:
        got = g.sir(1.0, 1.0, seed=12, n_sims=20, profile=True)
    want = oracle.sir(rp, ci, 1.0, 1.0, seed=12, n_sims=20)
    compare(got, want, "BFS")
    # the infected set of one outbreak is the index case's component
    import scipy.sparse as sps
    from scipy.sparse.csgraph import connected_components
    n = rp.size - 1
    A = sps.csr_matrix((np.ones(ci.size), ci, rp), shape=(n, n))
    _, lab = connected_components(A, directed=False)
    comp_deg = np.bincount(lab, weights=deg)
    comp_size = np.bincount(lab)
    assert np.array_equal(got["size"], comp_size[lab[got["index"]]])
    assert got["work"][1] == int(got["size"].sum())
    assert got["work"][0] == int(comp_deg[lab[got["index"]]].sum())
    assert all(v >= 0 for v in got["phase_ms"].values()) and got["phase_ms"]["attempts"] > 0


def test_sir_two_batches():
    """More simulations than one batch holds (1024): the outcomes and the
    spreading-power sums continue across the batch boundary."""
    rp, ci = gen.erdos_renyi(600, 0.01, 21)
    with efgpu.Graph(rp, ci) as g:
        got = g.sir(0.3, 0.3, seed=99, n_sims=1500)
    compare(got, oracle.sir(rp, ci, 0.3, 0.3, seed=99, n_sims=1500), "1500 simulations")
    glob = got["size"] >= 150
    sys.stderr.write(f"[sir] ER 600: {int(glob.sum())} global of 1500\n")
    assert 0 < glob[:1024].sum() and 0 < glob[1024:].sum()


def test_sir_t_max_and_edge_cases():
    rp, ci = gen.watts_strogatz(3000, 6, 0.1, 12)
    with efgpu.Graph(rp, ci) as g:
        cut = g.sir(0.4, 0.2, seed=5, n_sims=40, t_max=6)
        zero = g.sir(0.4, 0.2, seed=5, n_sims=40, t_max=0)
        none = g.sir(0.4, 0.2, seed=5, n_sims=0)
        dead = g.sir(0.0, 1.0, seed=5, n_sims=10)
    compare(cut, oracle.sir(rp, ci, 0.4, 0.2, seed=5, n_sims=40, t_max=6), "t_max = 6")
    assert np.all(cut["t_end"] <= 6)
    compare(zero, oracle.sir(rp, ci, 0.4, 0.2, seed=5, n_sims=40, t_max=0), "t_max = 0")
    assert np.all(zero["size"] == 1) and np.all(zero["t_end"] == 0)
    assert none["index"].size == 0 and not none["sp_sum"].any()
    # beta = 0, mu = 1: the index case recovers in the first step, infecting nobody
    assert np.all(dead["size"] == 1) and np.all(dead["t_end"] == 1)
    assert np.array_equal(dead["index"], cut["index"][:10])
    # isolated nodes and a graph with one node
    rp1, ci1 = gen.from_edges(5, [0], [1])
    with efgpu.Graph(rp1, ci1) as g:
        got = g.sir(1.0, 0.5, seed=3, n_sims=30)
    compare(got, oracle.sir(rp1, ci1, 1.0, 0.5, seed=3, n_sims=30), "K2 + isolated")
    with efgpu.Graph(np.zeros(2, np.int32), np.zeros(0, np.int32)) as g:
        got = g.sir(0.5, 0.5, seed=1, n_sims=4)
    assert np.all(got["index"] == 0) and np.all(got["size"] == 1)
    assert np.all(got["inf_count"] == 4)  # 1 >= ceil(1 / 4): every outbreak is global
