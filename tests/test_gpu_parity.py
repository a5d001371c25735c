"""Parity of the HIP path with the CPU oracle (needs an MI355X).

Every case calls the library through its C-ABI (efgpu binding) and compares,
element by element, with the oracle on the same seeded input:
  * N and D bit-exact;
  * EF within 1e-9 relative in FP64 mode and 1e-5 relative in FP32C mode
    (an oracle EF of exactly 0 must come back as exactly 0).
At the full R-MAT scale-22 size the oracle computes a stratified sample of
seeds, and properties that hold at any size are checked on every node.
"""
import functools
import itertools
import math
import sys

import numpy as np
import pytest

import oracle
from paper_2306_00606_amd import efgpu, gen
from tests import efref

pytestmark = pytest.mark.gpu

REL = {"fp64": 1e-9, "fp32c": 1e-5}
COMBOS = [(a, p) for a in ("cluster", "per_seed") for p in ("fp64", "fp32c")]


@pytest.fixture(autouse=True)
def _announce(request):
    sys.stderr.write(f"\n[gpu case] {request.node.nodeid}\n")
    sys.stderr.flush()
    yield


def assert_parity(ef, D, N, oN, oD, oE, prec, what=""):
    assert np.array_equal(N, oN), f"{what}: N differs at {np.flatnonzero(N != oN)[:10]}"
    assert np.array_equal(D, oD), f"{what}: D differs at {np.flatnonzero(D != oD)[:10]}"
    err = np.abs(ef - oE)
    bound = REL[prec] * np.abs(oE)
    bad = np.flatnonzero(err > bound)
    assert bad.size == 0, (f"{what} {prec}: {bad.size} EF outside tolerance, worst rel "
                           f"{np.max(err[bad] / np.maximum(np.abs(oE[bad]), 1e-300)):.3e} "
                           f"at node {bad[:5]} gpu {ef[bad[:5]]} oracle {oE[bad[:5]]}")
    assert not np.any(np.signbit(ef)), "negative zero or negative EF"
    rel = err[oE > 0] / oE[oE > 0]
    return float(rel.max()) if rel.size else 0.0


def run_all(rp, ci, algo, prec, seeds=None, validate=True):
    with efgpu.Graph(rp, ci, validate=validate) as g:
        return g.compute(algo=algo, prec=prec, seeds=seeds)


@functools.lru_cache(maxsize=None)
def oracle_all(name):
    rp, ci = GRAPHS[name]()
    return oracle.ef(rp, ci, threads=8)


GRAPHS = {
    "er1000_s1": lambda: gen.er_1000(1),
    "er1000_s7": lambda: gen.er_1000(7),
    "ba5000_m20": lambda: gen.barabasi_albert(5000, 20, 3),
    "rmat13_ef16": lambda: gen.rmat(13, 16, 5, perm_seed=6),
    "ws3000": lambda: gen.watts_strogatz(3000, 10, 0.1, 2),
    "cm4000": lambda: gen.config_model(4000, 2.1, 9),
}


# ---------------------------------------------------------------------------
PINS = efref.load_pins(efref.__file__.replace("efref.py", "golden/ef_pins.txt"))


@pytest.mark.parametrize("algo,prec", COMBOS)
def test_golden_pins(algo, prec):
    for pin in PINS:
        src, dst = efref.pin_graph(pin)
        rp, ci = gen.from_edges(pin["n"], src, dst)
        ef, D, N = run_all(rp, ci, algo, prec)
        s = pin["node"]
        assert (int(N[s]), int(D[s])) == (pin["N"], pin["D"]), pin["name"]
        want = efref.eval_pin_expr(pin["expr"])
        assert abs(ef[s] - want) <= REL[prec] * abs(want), (pin["name"], ef[s], want)


@pytest.mark.parametrize("algo,prec", COMBOS)
def test_every_graph_up_to_5_nodes(algo, prec):
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
    ef, D, N = run_all(rp, ci, algo, prec)
    oN, oD, oE = oracle.ef(rp, ci)
    assert_parity(ef, D, N, oN, oD, oE, prec, "all graphs n<=5")


@pytest.mark.parametrize("name", sorted(GRAPHS))
@pytest.mark.parametrize("algo,prec", COMBOS)
def test_random_graphs_all_nodes(name, algo, prec):
    rp, ci = GRAPHS[name]()
    ef, D, N = run_all(rp, ci, algo, prec)
    oN, oD, oE = oracle_all(name)
    worst = assert_parity(ef, D, N, oN, oD, oE, prec, name)
    sys.stderr.write(f"[parity] {name} {algo} {prec} max rel err {worst:.3e}\n")


def test_config1_er1000_seeds_1_to_20():
    for seed in range(1, 21):
        rp, ci = gen.er_1000(seed)
        oN, oD, oE = oracle.ef(rp, ci)
        for algo, prec in COMBOS:
            ef, D, N = run_all(rp, ci, algo, prec)
            assert_parity(ef, D, N, oN, oD, oE, prec, f"er1000 seed {seed}")


def hub_graph():
    """A hub of degree 3000 (two super-blocks, ragged; per-seed 16-wavefront bin),
    a second hub of degree 1500 sharing neighbours with it, on an ER
    background: many triangles through the hubs."""
    rs = np.random.default_rng(11)
    n = 6000
    src = [np.zeros(3000, np.int32), np.full(1500, 1, np.int32)]
    dst = [np.arange(2, 3002, dtype=np.int32), rs.choice(np.arange(2, n), 1500, replace=False).astype(np.int32)]
    e = rs.integers(0, n, size=(20000, 2)).astype(np.int32)
    src.append(e[:, 0])
    dst.append(e[:, 1])
    return gen.from_edges(n, np.concatenate(src), np.concatenate(dst))


@pytest.mark.parametrize("algo,prec", COMBOS)
def test_hub_graph(algo, prec):
    rp, ci = hub_graph()
    ef, D, N = run_all(rp, ci, algo, prec)
    oN, oD, oE = oracle.ef(rp, ci, threads=8)
    assert_parity(ef, D, N, oN, oD, oE, prec, "hub graph")


def table_edge_graph():
    """Hub H = 0 of degree 9000 and centre C = 1 of degree exactly 2048: C's
    neighbours in degree order end with H, so C's last 64-column block is full
    and holds a degree above the score table's reach (those tiles take the
    log), while its other tiles and all of H's read the table; some of C's
    neighbours are linked in pairs (triangles through C and H)."""
    rs = np.random.default_rng(7)
    n = 9100
    hub = np.arange(2, 9002, dtype=np.int32)                      # H's 9000 neighbours, with C
    hub[-1] = 1
    cn = rs.choice(np.arange(2, 9002), 2047, replace=False).astype(np.int32)
    pairs = cn[:600].reshape(-1, 2)
    e = rs.integers(9002, n, size=(300, 2)).astype(np.int32)
    src = np.concatenate([np.zeros(9000, np.int32), np.ones(2047, np.int32), pairs[:, 0], e[:, 0]])
    dst = np.concatenate([hub, cn, pairs[:, 1], e[:, 1]])
    return gen.from_edges(n, src, dst)


@pytest.mark.parametrize("prec", ["fp32c", "fp64"])
def test_score_table_and_log_tiles(prec):
    rp, ci = table_edge_graph()
    deg = np.diff(rp)
    assert deg[0] == 9000 and deg[1] == 2048
    ef, D, N = run_all(rp, ci, "cluster", prec)
    oN, oD, oE = oracle.ef(rp, ci, threads=8)
    assert_parity(ef, D, N, oN, oD, oE, prec, "score table edge")


def short_superblock_graph():
    """Centres whose last super-block of 1024 neighbours holds few 64-column
    blocks: degrees 1025 (one ragged block), 1088 (one full block), 1152 (two
    full), 1300 (five, ragged), 2100 (three super-blocks, the last one ragged
    block) and 4160 (five, the last one full block), so that up to 16
    wavefronts share a column block in one round of the super-tile loop. Each
    centre is linked to hub H = 0 (degree about 9000), whose degree puts the
    tiles holding it beyond the score table; random edges close triangles."""
    rs = np.random.default_rng(29)
    n = 12000
    degs = [1025, 1088, 1152, 1300, 2100, 4160]
    src = [np.zeros(9000, np.int32)]
    dst = [np.arange(12, 9012, dtype=np.int32)]
    for c, k in enumerate(degs, start=1):
        others = rs.choice(np.arange(12, n), k - 1, replace=False).astype(np.int32)
        src.append(np.full(k, c, np.int32))
        dst.append(np.concatenate([[0], others]).astype(np.int32))
    e = rs.integers(12, n, size=(3000, 2)).astype(np.int32)
    src.append(e[:, 0])
    dst.append(e[:, 1])
    return gen.from_edges(n, np.concatenate(src), np.concatenate(dst)), degs


@pytest.mark.parametrize("prec", ["fp32c", "fp64"])
def test_short_last_superblocks(prec):
    (rp, ci), degs = short_superblock_graph()
    deg = np.diff(rp)
    assert deg[1:7].tolist() == degs and deg[0] == 9006
    ef, D, N = run_all(rp, ci, "cluster", prec)
    oN, oD, oE = oracle.ef(rp, ci, threads=8)
    assert_parity(ef, D, N, oN, oD, oE, prec, "short last super-blocks")


def test_selected_seeds_with_duplicates():
    rp, ci = hub_graph()
    seeds = np.array([0, 1, 5, 0, 5999, 17, 1, 2, 3001], np.int32)
    oN, oD, oE = oracle.ef(rp, ci, seeds=seeds)
    with efgpu.Graph(rp, ci) as g:
        for prec in ("fp64", "fp32c"):
            ef, D, N = g.compute(algo="cluster", prec=prec, seeds=seeds)
            assert_parity(ef, D, N, oN, oD, oE, prec, "selected seeds")


def test_work_lists_kept_across_calls():
    """A handle keeps the pair loop's work lists of a whole-graph call; calls
    that bin a seed subset in between, and either formulation or precision
    after them, still give the results of a fresh handle (whole-graph
    cluster-centric calls bit for bit)."""
    rp, ci = hub_graph()
    seeds = np.array([0, 1, 5, 17, 3001], np.int32)
    with efgpu.Graph(rp, ci) as fresh:
        ref32 = fresh.compute(algo="cluster", prec="fp32c")
    with efgpu.Graph(rp, ci) as fresh:
        ref64 = fresh.compute(algo="cluster", prec="fp64")
    with efgpu.Graph(rp, ci) as g:
        runs = [("cluster", "fp32c", None), ("cluster", "fp32c", seeds), ("cluster", "fp32c", None),
                ("per_seed", "fp64", None), ("cluster", "fp64", None), ("cluster", "fp64", seeds),
                ("cluster", "fp32c", None)]
        for algo, prec, sd in runs:
            got = g.compute(algo=algo, prec=prec, seeds=sd)
            ref = ref32 if prec == "fp32c" else ref64
            idx = slice(None) if sd is None else seeds
            assert np.array_equal(got[1], ref[1][idx]) and np.array_equal(got[2], ref[2][idx])
            if algo == "cluster" and sd is None:
                assert np.array_equal(got[0], ref[0]), (algo, prec)
            else:  # a seed subset runs the per-seed formulation
                tol = 1e-5 if prec == "fp32c" else 1e-9
                assert np.allclose(got[0], ref[0][idx], rtol=tol, atol=0), (algo, prec)


def test_per_seed_equals_cluster_bitexact_integers_and_determinism():
    rp, ci = gen.rmat(14, 12, 21, perm_seed=4)
    with efgpu.Graph(rp, ci) as g:
        for prec in ("fp64", "fp32c"):
            e1, D1, N1 = g.compute(algo="cluster", prec=prec)
            e2, D2, N2 = g.compute(algo="per_seed", prec=prec)
            assert np.array_equal(D1, D2) and np.array_equal(N1, N2)
            e3, D3, N3 = g.compute(algo="cluster", prec=prec)
            assert np.array_equal(e1.view(np.int64), e3.view(np.int64)), "not reproducible"
            e4, _, _ = g.compute(algo="per_seed", prec=prec)
            assert np.array_equal(e2.view(np.int64), e4.view(np.int64)), "not reproducible"


def test_device_outputs_and_stream():
    torch = pytest.importorskip("torch")
    rp, ci = gen.rmat(12, 8, 2, perm_seed=3)
    oN, oD, oE = oracle.ef(rp, ci)
    dev = torch.device("cuda:0")
    rp_t = torch.from_numpy(rp).to(dev)
    ci_t = torch.from_numpy(ci).to(dev)
    with efgpu.Graph(rp_t, ci_t, validate=True) as g:
        n = rp.size - 1
        ef = torch.empty(n, dtype=torch.float64, device=dev)
        D = torch.empty(n, dtype=torch.int64, device=dev)
        N = torch.empty(n, dtype=torch.int64, device=dev)
        g.compute(algo="cluster", prec="fp32c", out=(ef, D, N))
        torch.cuda.synchronize()
        assert_parity(ef.cpu().numpy(), D.cpu().numpy(), N.cpu().numpy(), oN, oD, oE, "fp32c")
        seeds = np.array([3, 3, 100, 7], np.int32)
        efs = torch.empty(4, dtype=torch.float64, device=dev)
        g.compute(algo="per_seed", prec="fp64", seeds=seeds, out=(efs, None, None))
        torch.cuda.synchronize()
        assert np.allclose(efs.cpu().numpy(), oE[seeds], rtol=1e-9, atol=0)


def test_edge_cases():
    # no nodes
    with efgpu.Graph(np.zeros(1, np.int32), np.zeros(0, np.int32)) as g:
        ef, D, N = g.compute()
        assert ef.size == 0
    # only isolated nodes, and K2 components
    for rp, ci in (gen.from_edges(5, [], []), gen.from_edges(6, [0, 2, 4], [1, 3, 5])):
        for algo, prec in COMBOS:
            ef, D, N = run_all(rp, ci, algo, prec)
            assert np.all(ef == 0.0) and np.all(D == 0) and np.all(N == 0)
            assert not np.any(np.signbit(ef))
    # a seed list naming an out-of-range node is rejected
    rp, ci = gen.er_1000(1)
    with efgpu.Graph(rp, ci) as g:
        with pytest.raises(efgpu.EFError) as ei:
            g.compute(seeds=[0, 1000])
        assert ei.value.name == "EF_ERR_RANGE"
    # malformed input is rejected on load, also without the host validation
    # (the up-arc count of an asymmetric CSR is checked before it is used)
    for validate in (True, False):
        with pytest.raises(efgpu.EFError) as ei:
            efgpu.Graph(np.array([0, 1, 1], np.int32), np.array([1], np.int32), validate=validate)
        assert ei.value.name == "EF_ERR_NOT_SYMMETRIC"
    with pytest.raises(efgpu.EFError) as ei:
        efgpu.Graph(np.array([0, 2, 2, 2], np.int32), np.array([1, 2], np.int32), validate=False)
    assert ei.value.name == "EF_ERR_NOT_SYMMETRIC"


def dense_core_graph():
    """A core of 2300 nodes with edge probability 0.97 on a sparse periphery of
    3000 nodes: the lowest-ranked core nodes have more than 2048 members of
    higher rank (triangles listed from global memory), the rest of the core
    513..2048 (16-wavefront workgroups, several segment chunks)."""
    rs = np.random.default_rng(5)
    nc, n = 2300, 5300
    iu = np.triu_indices(nc, 1)
    keep = rs.random(iu[0].size) < 0.97
    src = [iu[0][keep].astype(np.int32)]
    dst = [iu[1][keep].astype(np.int32)]
    e = rs.integers(0, n, size=(12000, 2)).astype(np.int32)
    src.append(e[:, 0])
    dst.append(e[:, 1])
    return gen.from_edges(n, np.concatenate(src), np.concatenate(dst))


@pytest.mark.parametrize("prec", ["fp64", "fp32c"])
def test_dense_core_long_lists(prec):
    rp, ci = dense_core_graph()
    n = rp.size - 1
    deg = np.diff(rp).astype(np.int64)
    ef, D, N = run_all(rp, ci, "cluster", prec)
    src = np.repeat(np.arange(n), deg)
    A = np.bincount(src, weights=deg[ci], minlength=n).astype(np.int64)
    assert np.array_equal(N, deg * deg - 2 * deg + A)
    rng = np.random.default_rng(3)
    core = np.argsort(deg)[::-1][:2300]
    seeds = np.unique(np.concatenate([np.sort(core)[:12], rng.choice(core, 12, replace=False),
                                      rng.choice(np.arange(2300, n), 12, replace=False)]))
    seeds = seeds.astype(np.int32)
    oN, oD, oE = oracle.ef(rp, ci, seeds=seeds, threads=16)
    worst = assert_parity(ef[seeds], D[seeds], N[seeds], oN, oD, oE, prec, "dense core")
    sys.stderr.write(f"[parity] dense core {prec} {seeds.size} seeds max rel err {worst:.3e}\n")


@pytest.mark.parametrize("algo,prec", [("cluster", "fp32c"), ("cluster", "fp64"),
                                       ("per_seed", "fp32c")])
def test_config2_ba_1m_all_nodes(algo, prec):
    rp, ci = gen.ba_1m()
    ef, D, N = run_all(rp, ci, algo, prec, validate=False)
    oN, oD, oE = oracle_ba()
    worst = assert_parity(ef, D, N, oN, oD, oE, prec, "BA 1M")
    sys.stderr.write(f"[parity] BA 1M {algo} {prec} max rel err {worst:.3e}\n")


@functools.lru_cache(maxsize=None)
def oracle_ba():
    rp, ci = gen.ba_1m()
    return oracle.ef(rp, ci, threads=16)


def rmat22_sample(rp, deg, rng):
    """Stratified seeds: per degree bin up to 40 random nodes, plus the three
    largest nodes of degree <= 20000 (the oracle's per-seed cost is about
    k^2 + sum of neighbour degrees)."""
    bins = [0, 1, 2, 4, 16, 64, 256, 1024, 4096, 16384]
    out = []
    for lo, hi in zip(bins, bins[1:] + [20001]):
        idx = np.flatnonzero((deg >= lo) & (deg < hi))
        if idx.size:
            out.extend(rng.choice(idx, min(40, idx.size), replace=False).tolist())
    big = np.flatnonzero(deg <= 20000)
    out.extend(big[np.argsort(deg[big])[-3:]].tolist())
    return np.array(sorted(set(out)), np.int32)


def test_config3_rmat22_full_size_sampled():
    rp, ci = gen.rmat_22()
    n = rp.size - 1
    deg = np.diff(rp).astype(np.int64)
    with efgpu.Graph(rp, ci, validate=False) as g:
        ef, D, N = g.compute(algo="cluster", prec="fp32c")
        st = g.stats()
    sys.stderr.write(f"[rmat22] promoted {st['promoted']} fp64-finalised {st['fp64_finalized']}\n")
    # properties on every node: N closed form, sum rule, entropy bounds
    src = np.repeat(np.arange(n), deg)
    A = np.bincount(src, weights=deg[ci], minlength=n).astype(np.int64)
    assert np.array_equal(N, deg * deg - 2 * deg + A)
    assert int(N.sum()) == 4 * int((deg * (deg - 1) // 2).sum())
    ok = N > 1
    assert np.all(ef >= 0) and np.all(ef[~ok] == 0)
    assert np.all(ef[ok] <= np.log(N[ok].astype(np.float64)) * (1 + 1e-6))
    seeds = rmat22_sample(rp, deg, np.random.default_rng(22))
    oN, oD, oE = oracle.ef(rp, ci, seeds=seeds, threads=16)
    worst = assert_parity(ef[seeds], D[seeds], N[seeds], oN, oD, oE, "fp32c", "R-MAT 22 sample")
    sys.stderr.write(f"[parity] R-MAT 22 sample of {seeds.size}: max rel err {worst:.3e}\n")


@pytest.mark.parametrize("prec", ["fp64", "fp32c"])
def test_topk_matches_oracle(prec):
    """Top-k: EF descending, ties by id ascending. Compared with the oracle as a
    set, nodes whose oracle EF lies within the tolerance of the k-th value being
    interchangeable; the returned order must follow the returned EF."""
    rp, ci = GRAPHS["rmat13_ef16"]()
    oN, oD, oE = oracle_all("rmat13_ef16")
    tol = REL[prec]
    with efgpu.Graph(rp, ci) as g:
        ef_all, _, _ = g.compute(algo="cluster", prec=prec)
        for k in (1, 10, 100, 1000):
            nodes, ef = g.topk(k, prec=prec)
            assert nodes.size == k and np.array_equal(ef, ef_all[nodes])
            # order: descending EF, ties by id ascending
            for a, b, ea, eb in zip(nodes[:-1], nodes[1:], ef[:-1], ef[1:]):
                assert ea > eb or (ea == eb and a < b)
            kth = np.sort(oE)[::-1][k - 1]
            sure_in = np.flatnonzero(oE > kth * (1 + 2 * tol))
            assert set(sure_in.tolist()) <= set(nodes.tolist())
            assert np.all(oE[nodes] >= kth * (1 - 2 * tol))
        # k = 0 and k = n
        n = rp.size - 1
        nodes, ef = g.topk(n, prec=prec)
        assert np.array_equal(np.sort(nodes), np.arange(n))
        with pytest.raises(efgpu.EFError):
            g.topk(n + 1)
