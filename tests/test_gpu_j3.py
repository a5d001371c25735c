"""Parity of the three-event Expected Force (ef_compute_j3) with the CPU
oracle (needs an MI355X).

N and D bit-exact; EF within 1e-9 relative in FP64 and 1e-5 relative in FP32C
(an oracle EF of exactly 0 must come back as exactly 0). On larger graphs the
oracle takes a sample of seeds, and the identity N_3(s) = D_2(s) (the
three-event count equals the two-event degree sum) is checked on every node
against the library's own two-event result.
"""
import functools
import itertools
import sys

import numpy as np
import pytest

import oracle
from paper_2306_00606_amd import efgpu, gen
from tests import efref

pytestmark = pytest.mark.gpu

REL = {"fp64": 1e-9, "fp32c": 1e-5}
PRECS = ["fp64", "fp32c"]


@pytest.fixture(autouse=True)
def _announce(request):
    sys.stderr.write(f"\n[gpu case] {request.node.nodeid}\n")
    sys.stderr.flush()
    yield


def assert_parity(ef, D, N, oN, oD, oE, prec, what=""):
    assert np.array_equal(N, oN), f"{what}: N differs at {np.flatnonzero(N != oN)[:10]}"
    assert np.array_equal(D, oD), f"{what}: D differs at {np.flatnonzero(D != oD)[:10]}"
    err = np.abs(ef - oE)
    bad = np.flatnonzero(err > REL[prec] * np.abs(oE))
    assert bad.size == 0, (f"{what} {prec}: {bad.size} EF outside tolerance at {bad[:5]}: "
                           f"gpu {ef[bad[:5]]} oracle {oE[bad[:5]]}")
    assert not np.any(np.signbit(ef)), "negative zero or negative EF"


GRAPHS = {
    "er1000": lambda: gen.er_1000(3),
    "ba3000_m6": lambda: gen.barabasi_albert(3000, 6, 4),
    "rmat11_ef8": lambda: gen.rmat(11, 8, 2, perm_seed=5),
    "ws2000": lambda: gen.watts_strogatz(2000, 8, 0.2, 3),
    "cm2000": lambda: gen.config_model(2000, 2.4, 7),
}


@functools.lru_cache(maxsize=None)
def oracle3(name):
    rp, ci = GRAPHS[name]()
    return oracle.ef(rp, ci, threads=16, j=3)


PINS = efref.load_pins(efref.__file__.replace("efref.py", "golden/ef3_pins.txt"))


@pytest.mark.parametrize("prec", PRECS)
def test_golden_pins_j3(prec):
    for pin in PINS:
        src, dst = efref.pin_graph(pin)
        rp, ci = gen.from_edges(pin["n"], src, dst)
        with efgpu.Graph(rp, ci) as g:
            ef, D, N = g.compute(prec=prec, j=3)
        s = pin["node"]
        assert (int(N[s]), int(D[s])) == (pin["N"], pin["D"]), pin["name"]
        want = efref.eval_pin_expr(pin["expr"])
        assert abs(ef[s] - want) <= REL[prec] * abs(want), (pin["name"], ef[s], want)


@pytest.mark.parametrize("prec", PRECS)
def test_every_graph_up_to_5_nodes_j3(prec):
    src, dst, off = [], [], 0
    for n in range(1, 6):
        pairs = list(itertools.combinations(range(n), 2))
        for mask in range(1 << len(pairs)):
            for i, (u, v) in enumerate(pairs):
                if mask >> i & 1:
                    src.append(off + u)
                    dst.append(off + v)
            off += n
    rp, ci = gen.from_edges(off, np.array(src, np.int32), np.array(dst, np.int32))
    with efgpu.Graph(rp, ci) as g:
        ef, D, N = g.compute(prec=prec, j=3)
    oN, oD, oE = oracle.ef(rp, ci, j=3)
    assert_parity(ef, D, N, oN, oD, oE, prec, "all graphs n<=5")


@pytest.mark.parametrize("name", sorted(GRAPHS))
@pytest.mark.parametrize("prec", PRECS)
def test_graphs_all_nodes_j3(name, prec):
    rp, ci = GRAPHS[name]()
    with efgpu.Graph(rp, ci) as g:
        ef, D, N = g.compute(prec=prec, j=3)
        st = g.stats()
    oN, oD, oE = oracle3(name)
    assert_parity(ef, D, N, oN, oD, oE, prec, name)
    sys.stderr.write(f"[j3] {name} {prec}: recomputed in FP64 {st['promoted']}\n")


def test_selected_seeds_duplicates_and_device_outputs_j3():
    torch = pytest.importorskip("torch")
    rp, ci = GRAPHS["rmat11_ef8"]()
    oN, oD, oE = oracle3("rmat11_ef8")
    seeds = np.array([5, 0, 5, 2047, 17, 0, 1000], np.int32)
    dev = torch.device("cuda:0")
    with efgpu.Graph(rp, ci) as g:
        for prec in PRECS:
            ef, D, N = g.compute(prec=prec, seeds=seeds, j=3)
            assert_parity(ef, D, N, oN[seeds], oD[seeds], oE[seeds], prec, "seeds")
        n = rp.size - 1
        e_t = torch.empty(n, dtype=torch.float64, device=dev)
        D_t = torch.empty(n, dtype=torch.int64, device=dev)
        N_t = torch.empty(n, dtype=torch.int64, device=dev)
        g.compute(prec="fp32c", out=(e_t, D_t, N_t), j=3)
        torch.cuda.synchronize()
        assert_parity(e_t.cpu().numpy(), D_t.cpu().numpy(), N_t.cpu().numpy(), oN, oD, oE,
                      "fp32c", "device outputs")
        es = torch.empty(seeds.size, dtype=torch.float64, device=dev)
        g.compute(prec="fp64", seeds=seeds, out=(es, None, None), j=3)
        torch.cuda.synchronize()
        assert np.allclose(es.cpu().numpy(), oE[seeds], rtol=1e-9, atol=0)


def test_larger_graph_identity_and_sample_j3():
    """BA n = 200,000, m = 5: N_3 = D_2 on every node against the two-event
    result, reproducible bits, and the oracle on a sample of seeds whose
    sequence count stays below 2e8."""
    rp, ci = gen.barabasi_albert(200_000, 5, 11)
    with efgpu.Graph(rp, ci, validate=False) as g:
        ef3, D3, N3 = g.compute(prec="fp32c", j=3)
        ef3b, _, _ = g.compute(prec="fp32c", j=3)
        _, D2, N2 = g.compute(algo="cluster", prec="fp32c")
        ef64, D64, N64 = g.compute(prec="fp64", j=3)
    assert np.array_equal(N3, D2), "three-event count differs from the two-event degree sum"
    assert np.array_equal(ef3.view(np.int64), ef3b.view(np.int64)), "not reproducible"
    assert np.array_equal(D3, D64) and np.array_equal(N3, N64)
    assert np.all(ef3 >= 0) and np.all(ef3 <= np.log(np.maximum(N3, 1).astype(np.float64)) + 1e-9)
    rng = np.random.default_rng(5)
    small = np.flatnonzero(N3 < 2e8)
    big = small[np.argsort(N3[small])[-4:]]
    seeds = np.unique(np.concatenate([rng.choice(small, 40, replace=False), big])).astype(np.int32)
    oN, oD, oE = oracle.ef(rp, ci, seeds=seeds, threads=16, j=3)
    assert_parity(ef3[seeds], D3[seeds], N3[seeds], oN, oD, oE, "fp32c", "BA 200k sample")
    assert_parity(ef64[seeds], D64[seeds], N64[seeds], oN, oD, oE, "fp64", "BA 200k sample")


def test_edge_cases_j3():
    with efgpu.Graph(np.zeros(1, np.int32), np.zeros(0, np.int32)) as g:
        ef, D, N = g.compute(j=3)
        assert ef.size == 0
    # isolated nodes, K2 and P3 components: fewer than three events, N = 0
    rp, ci = gen.from_edges(9, [0, 2, 5, 6], [1, 3, 6, 7])
    with efgpu.Graph(rp, ci) as g:
        for prec in PRECS:
            ef, D, N = g.compute(prec=prec, j=3)
            assert np.all(ef == 0.0) and np.all(D == 0) and np.all(N == 0)
            assert not np.any(np.signbit(ef))
    # a star too large for int64 sums is rejected before any kernel runs
    L = 200_000
    rp, ci = gen.from_edges(L + 1, np.zeros(L, np.int32), np.arange(1, L + 1, dtype=np.int32))
    with efgpu.Graph(rp, ci) as g:
        with pytest.raises(efgpu.EFError) as ei:
            g.compute(j=3)
        assert ei.value.name == "EF_ERR_OVERFLOW"


def two_hub_graph():
    """Hubs 0 and 1 (adjacent, 4200 leaves each, some leaves of 1 also joined
    to 0, and 100 leaf-leaf edges across): the first events 0 -> 1 and
    1 -> 0 have lists longer than 8192 (merge path), the leaves' first events
    lists of about 4200 (the largest union bin)."""
    L = 4200
    src = [0] + [0] * L + [1] * L + [0] * 50
    dst = [1] + list(range(2, 2 + L)) + list(range(2 + L, 2 + 2 * L)) + list(range(2 + L, 52 + L))
    src += list(range(2, 102))
    dst += list(range(2 + L, 102 + L))
    return gen.from_edges(2 + 2 * L, np.array(src, np.int32), np.array(dst, np.int32))


def test_two_hubs_merge_path_j3():
    rp, ci = two_hub_graph()
    with efgpu.Graph(rp, ci) as g:
        e32, D32, N32 = g.compute(prec="fp32c", j=3)
        e64, D64, N64 = g.compute(prec="fp64", j=3)
        _, D2, _ = g.compute(algo="cluster", prec="fp64")
    assert np.array_equal(N32, D2) and np.array_equal(N64, D2)
    assert np.array_equal(D32, D64)
    ok = e64 > 0
    assert np.all(np.abs(e32[ok] - e64[ok]) <= 1e-5 * e64[ok]) and np.all(e32[~ok] == 0)
    seeds = np.array([2, 3, 60, 150, 2 + 4200, 2 + 4200 + 10, 2 + 4200 + 120, 8401], np.int32)
    oN, oD, oE = oracle.ef(rp, ci, seeds=seeds, threads=16, j=3)
    assert_parity(e64[seeds], D64[seeds], N64[seeds], oN, oD, oE, "fp64", "two hubs")
    assert_parity(e32[seeds], D32[seeds], N32[seeds], oN, oD, oE, "fp32c", "two hubs")
