"""The degree-class aggregated cluster-centric variant (EF_ALGO_CLUSTER_AGG)
against the CPU oracle (needs an MI355X). Centres of degree > 1024 take the
aggregated path; one with more than 4096 distinct neighbour degrees falls back
to the super-tile pair loop inside the same call."""
import functools
import sys

import numpy as np
import pytest

import oracle
from paper_2306_00606_amd import efgpu, gen
from tests import test_gpu_parity as P

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _announce(request):
    sys.stderr.write(f"\n[gpu case] {request.node.nodeid}\n")
    sys.stderr.flush()
    yield


@pytest.mark.parametrize("prec", ["fp64", "fp32c"])
def test_agg_hub_graph(prec):
    rp, ci = P.hub_graph()
    ef, D, N = P.run_all(rp, ci, "cluster_agg", prec)
    oN, oD, oE = oracle.ef(rp, ci, threads=8)
    worst = P.assert_parity(ef, D, N, oN, oD, oE, prec, "hub graph (agg)")
    sys.stderr.write(f"[agg] hub graph {prec} max rel err {worst:.3e}\n")


@pytest.mark.parametrize("prec", ["fp64", "fp32c"])
def test_agg_ba_1m_all_nodes(prec):
    rp, ci = gen.ba_1m()
    ef, D, N = P.run_all(rp, ci, "cluster_agg", prec, validate=False)
    oN, oD, oE = P.oracle_ba()
    worst = P.assert_parity(ef, D, N, oN, oD, oE, prec, "BA 1M (agg)")
    sys.stderr.write(f"[agg] BA 1M {prec} max rel err {worst:.3e}\n")


def test_agg_rmat22_sampled_and_reproducible():
    rp, ci = gen.rmat_22()
    deg = np.diff(rp).astype(np.int64)
    with efgpu.Graph(rp, ci, validate=False) as g:
        ef, D, N = g.compute(algo="cluster_agg", prec="fp32c")
        ef2, D2, N2 = g.compute(algo="cluster_agg", prec="fp32c")
        ec, Dc, Nc = g.compute(algo="cluster", prec="fp32c")
    assert np.array_equal(ef.view(np.int64), ef2.view(np.int64)), "not reproducible"
    assert np.array_equal(D, Dc) and np.array_equal(N, Nc)
    seeds = P.rmat22_sample(rp, deg, np.random.default_rng(22))
    oN, oD, oE = oracle.ef(rp, ci, seeds=seeds, threads=16)
    worst = P.assert_parity(ef[seeds], D[seeds], N[seeds], oN, oD, oE, "fp32c",
                            "R-MAT 22 sample (agg)")
    sys.stderr.write(f"[agg] R-MAT 22 sample of {seeds.size}: max rel err {worst:.3e}\n")


@functools.lru_cache(maxsize=None)
def many_degree_graph():
    """A hub (node 0) whose 4300 neighbours v_1..v_4300 have 4300 distinct
    degrees (v_i is also joined to i filler nodes), so the hub has more
    distinct neighbour degrees than the aggregated path holds and falls back;
    the 4400 fillers are big centres with many distinct neighbour degrees too."""
    rs = np.random.default_rng(5)
    m, nf = 4300, 4400
    n = 1 + m + nf
    src, dst = [], []
    v = np.arange(1, m + 1, dtype=np.int32)
    src.append(np.zeros(m, np.int32))
    dst.append(v)
    for i in range(1, m + 1):
        f = rs.choice(nf, size=i, replace=False).astype(np.int32) + 1 + m
        src.append(np.full(i, i, np.int32))
        dst.append(f)
    return gen.from_edges(n, np.concatenate(src), np.concatenate(dst))


def test_agg_fallback_many_distinct_degrees():
    rp, ci = many_degree_graph()
    deg = np.diff(rp)
    seeds = np.array([0, 1, 2, 100, 4300, 4301, 4302, 7000, int(np.argmax(deg[4301:])) + 4301],
                     np.int32)
    oN, oD, oE = oracle.ef(rp, ci, seeds=seeds, threads=16)
    with efgpu.Graph(rp, ci, validate=False) as g:
        for prec in ("fp64", "fp32c"):
            ef, D, N = g.compute(algo="cluster_agg", prec=prec)
            P.assert_parity(ef[seeds], D[seeds], N[seeds], oN, oD, oE, prec, "fallback (agg)")
            ec, Dc, Nc = g.compute(algo="cluster", prec=prec)
            assert np.array_equal(D, Dc) and np.array_equal(N, Nc)
            rel = np.abs(ef - ec) / np.maximum(np.abs(ec), 1e-300)
            assert np.all(rel[ec > 0] <= 2 * P.REL[prec]), float(rel.max())
