"""Full-size parity on the headline graph and on the per-seed formulation's
largest bin (needs an MI355X).

* R-MAT scale 22, edge factor 10: every formulation and precision runs on all
  4,194,304 nodes in the configuration the benchmark times, and is compared
  element by element with oracle values stored in ``golden/rmat22_oracle.txt``
  (written by ``golden/make_rmat22_golden.py`` from the CPU oracle alone). The
  stored seeds hold every node of degree above 20000, 40 nodes of degree
  8193..20000 (the per-seed bitmap bin) and a stratified sample.
  N and D bit-exact, EF within 1e-9 (FP64) and 1e-5 (FP32C) relative. On every
  node, per-seed N and D equal the cluster-centric ones bit for bit and the
  two EF agree within the tolerance.
* A graph with five seeds of degree 8193..20000 (the bitmap bin), checked on
  every node against the oracle, for both formulations and precisions, and as
  selected seeds with duplicates.
"""
import functools
import os
import sys

import numpy as np
import pytest

import oracle
from paper_2306_00606_amd import efgpu, gen

pytestmark = pytest.mark.gpu

REL = {"fp64": 1e-9, "fp32c": 1e-5}
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "rmat22_oracle.txt")


@pytest.fixture(autouse=True)
def _announce(request):
    sys.stderr.write(f"\n[gpu case] {request.node.nodeid}\n")
    sys.stderr.flush()
    yield


def load_golden():
    rows = []
    with open(GOLDEN) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            node, deg, groups, N, D, E = [x.strip() for x in line.split("|")]
            rows.append((int(node), int(deg), groups, int(N), int(D), float(E)))
    nodes = np.array([r[0] for r in rows], np.int64)
    return (nodes, np.array([r[1] for r in rows], np.int64), [r[2] for r in rows],
            np.array([r[3] for r in rows], np.int64), np.array([r[4] for r in rows], np.int64),
            np.array([r[5] for r in rows], np.float64))


def check(ef, D, N, oN, oD, oE, prec, what):
    assert np.array_equal(N, oN), f"{what}: N differs at {np.flatnonzero(N != oN)[:10]}"
    assert np.array_equal(D, oD), f"{what}: D differs at {np.flatnonzero(D != oD)[:10]}"
    err = np.abs(ef - oE)
    bad = np.flatnonzero(err > REL[prec] * np.abs(oE))
    assert bad.size == 0, (f"{what} {prec}: {bad.size} EF outside tolerance at {bad[:5]}: "
                           f"gpu {ef[bad[:5]]} oracle {oE[bad[:5]]}")
    assert not np.any(np.signbit(ef))
    pos = oE > 0
    return float((err[pos] / oE[pos]).max()) if pos.any() else 0.0


@functools.lru_cache(maxsize=None)
def rmat22():
    return gen.rmat_22()


@functools.lru_cache(maxsize=None)
def rmat22_cluster_fp32c():
    rp, ci = rmat22()
    with efgpu.Graph(rp, ci, validate=False) as g:
        return g.compute(algo="cluster", prec="fp32c")


def test_golden_file_matches_graph():
    rp, _ = rmat22()
    nodes, deg, groups, oN, _, _ = load_golden()
    assert np.array_equal(np.diff(rp)[nodes], deg)
    d = np.diff(rp)
    # every node above degree 20000 is stored, and the bitmap bin is present
    assert set(np.flatnonzero(d > 20000).tolist()) <= set(nodes.tolist())
    assert sum("big" in g for g in groups) == 40
    assert int(oN.max()) > 1 << 24


@pytest.mark.parametrize("algo,prec", [("cluster", "fp32c"), ("cluster", "fp64"),
                                       ("per_seed", "fp32c"), ("per_seed", "fp64")])
def test_rmat22_all_nodes_against_stored_oracle(algo, prec):
    rp, ci = rmat22()
    nodes, deg, groups, oN, oD, oE = load_golden()
    if (algo, prec) == ("cluster", "fp32c"):
        ef, D, N = rmat22_cluster_fp32c()
    else:
        with efgpu.Graph(rp, ci, validate=False) as g:
            ef, D, N = g.compute(algo=algo, prec=prec)
    worst = check(ef[nodes], D[nodes], N[nodes], oN, oD, oE, prec, f"R-MAT 22 {algo}")
    hub = deg > 20000
    whub = check(ef[nodes[hub]], D[nodes[hub]], N[nodes[hub]], oN[hub], oD[hub], oE[hub], prec,
                 "hubs")
    sys.stderr.write(f"[parity] R-MAT 22 {algo} {prec}: {nodes.size} stored seeds, max rel err "
                     f"{worst:.3e} (hubs {whub:.3e})\n")
    if algo == "per_seed":
        # every node: integers equal the cluster-centric formulation's bit for bit
        cef, cD, cN = rmat22_cluster_fp32c()
        assert np.array_equal(N, cN) and np.array_equal(D, cD)
        tol = REL["fp32c"] + REL[prec]
        rel = np.abs(ef - cef) / np.maximum(np.abs(cef), 1e-300)
        assert np.all((rel <= tol) | ((ef == 0) & (cef == 0))), (
            f"per-seed vs cluster EF: worst rel {rel.max():.3e} at {np.argmax(rel)}")


def test_rmat22_selected_hub_seeds():
    """Selected seeds always take the per-seed kernel: every stored hub and
    bitmap-bin seed, with a duplicate, in both precisions."""
    rp, ci = rmat22()
    nodes, deg, groups, oN, oD, oE = load_golden()
    pick = np.flatnonzero(deg > 8192)
    sel = np.concatenate([nodes[pick], nodes[pick[:3]]]).astype(np.int32)
    want = np.concatenate([pick, pick[:3]])
    with efgpu.Graph(rp, ci, validate=False) as g:
        for prec in ("fp32c", "fp64"):
            ef, D, N = g.compute(algo="per_seed", prec=prec, seeds=sel)
            check(ef, D, N, oN[want], oD[want], oE[want], prec, "selected hub seeds")


def bitmap_seed_graph():
    """Five seeds of degree 8193, 9000, 12000, 16384 and 20000 (above the
    per-seed kernel's LDS-hash limit of 8192, so their membership tests go
    through device bitmaps), linked in a ring, with random neighbourhoods that
    overlap, on a sparse random background of 40000 nodes."""
    rs = np.random.default_rng(8193)
    n = 40000
    hub_deg = [8193, 9000, 12000, 16384, 20000]
    h = len(hub_deg)
    src, dst = [], []
    for i, k in enumerate(hub_deg):
        src.append(np.full(k - 2, i, np.int32))
        dst.append(rs.choice(np.arange(h, n), k - 2, replace=False).astype(np.int32))
    src.append(np.arange(h, dtype=np.int32))
    dst.append(((np.arange(h) + 1) % h).astype(np.int32))
    e = rs.integers(h, n, size=(60000, 2)).astype(np.int32)
    src.append(e[:, 0])
    dst.append(e[:, 1])
    return gen.from_edges(n, np.concatenate(src), np.concatenate(dst))


@functools.lru_cache(maxsize=None)
def bitmap_oracle():
    rp, ci = bitmap_seed_graph()
    return oracle.ef(rp, ci, threads=8)


@pytest.mark.parametrize("algo,prec", [(a, p) for a in ("per_seed", "cluster")
                                       for p in ("fp32c", "fp64")])
def test_bitmap_bin_seeds_all_nodes(algo, prec):
    rp, ci = bitmap_seed_graph()
    deg = np.diff(rp)
    assert list(deg[:5]) == [8193, 9000, 12000, 16384, 20000]
    oN, oD, oE = bitmap_oracle()
    with efgpu.Graph(rp, ci) as g:
        ef, D, N = g.compute(algo=algo, prec=prec)
    worst = check(ef, D, N, oN, oD, oE, prec, f"bitmap graph {algo}")
    sys.stderr.write(f"[parity] bitmap graph {algo} {prec}: max rel err {worst:.3e}\n")


def test_bitmap_bin_selected_seeds_twice():
    """Selected seeds, duplicates included, twice on one handle: the second
    call reuses the bitmaps the first one left, which must come back clean."""
    rp, ci = bitmap_seed_graph()
    oN, oD, oE = bitmap_oracle()
    sel = np.array([4, 0, 17, 4, 3, 39999, 1, 2, 2, 5000], np.int32)
    with efgpu.Graph(rp, ci) as g:
        for prec in ("fp32c", "fp64", "fp32c"):
            ef, D, N = g.compute(algo="per_seed", prec=prec, seeds=sel)
            check(ef, D, N, oN[sel], oD[sel], oE[sel], prec, "selected bitmap seeds")
        ef, D, N = g.compute(algo="per_seed", prec="fp64", seeds=sel[::-1].copy())
        check(ef, D, N, oN[sel[::-1]], oD[sel[::-1]], oE[sel[::-1]], "fp64", "reversed")
