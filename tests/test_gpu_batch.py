"""Batched computation (disjoint union, captured HIP graph, tuned thresholds;
the phased design and the persistent kernel) against the oracle and against
one-graph-at-a-time computation (needs an MI355X)."""
import sys

import numpy as np
import pytest

import oracle
from paper_2306_00606_amd import efgpu, gen

pytestmark = pytest.mark.gpu

REL = {"fp64": 1e-9, "fp32c": 1e-5}


@pytest.fixture(autouse=True)
def _announce(request):
    sys.stderr.write(f"\n[gpu case] {request.node.nodeid}\n")
    sys.stderr.flush()
    yield


def small_batch():
    # the batch recipe at small sizes: WS and erased CM graphs of uneven size
    return gen.batch_512(seed0=77, count=24, n_lo=50, n_hi=3000)


@pytest.mark.parametrize("design", ["phased", "persistent"])
@pytest.mark.parametrize("prec", ["fp32c", "fp64"])
def test_batch_matches_oracle_and_single_graphs(prec, design):
    graphs = small_batch()
    with efgpu.Batch(graphs, validate=True) as b:
        ef, D, N = b.compute(prec=prec, design=design)
        st = b.stats()
        assert st["n_graphs"] == len(graphs) and st["n"] == ef.size
        for i, (rp, ci) in enumerate(graphs):
            sl = slice(int(b.node_off[i]), int(b.node_off[i + 1]))
            oN, oD, oE = oracle.ef(rp, ci)
            assert np.array_equal(N[sl], oN) and np.array_equal(D[sl], oD), i
            err = np.abs(ef[sl] - oE)
            assert np.all(err <= REL[prec] * np.abs(oE)), (i, float(err.max()))
            with efgpu.Graph(rp, ci) as g:
                e1, D1, N1 = g.compute(algo="cluster", prec=prec)
            assert np.array_equal(D1, D[sl]) and np.array_equal(N1, N[sl])
            assert np.all(np.abs(e1 - ef[sl]) <= REL[prec] * np.abs(oE))


@pytest.mark.parametrize("design", ["phased", "persistent"])
def test_graph_replays_match_eager(design):
    """Replay the captured graph several times, with unrelated eager work and
    synchronisations in between; every replay must equal the first result
    bit for bit."""
    torch = pytest.importorskip("torch")
    graphs = small_batch()
    other = gen.rmat(11, 8, 3, perm_seed=4)
    with efgpu.Batch(graphs) as b, efgpu.Graph(*other) as g:
        b.autotune("fp32c")
        ref = b.compute(prec="fp32c", design=design)
        dev = torch.device("cuda:0")
        ef_t = torch.empty(b.n, dtype=torch.float64, device=dev)
        D_t = torch.empty(b.n, dtype=torch.int64, device=dev)
        N_t = torch.empty(b.n, dtype=torch.int64, device=dev)
        for r in range(5):
            g.compute(algo="per_seed", prec="fp64")  # eager work on the same device
            torch.cuda.synchronize()
            ef_t.fill_(-1.0)
            b.compute(prec="fp32c", out=(ef_t, D_t, N_t), profile=(r == 4), design=design)
            torch.cuda.synchronize()
            assert np.array_equal(ef_t.cpu().numpy().view(np.int64), ref[0].view(np.int64)), r
            assert np.array_equal(D_t.cpu().numpy(), ref[1])
            assert np.array_equal(N_t.cpu().numpy(), ref[2])
        st = b.stats()
        assert st["replay_ms"] > 0
        assert 0 <= st["tuned_choice"] < 8 and 0 <= st["persist_choice"] < 8
        assert st["design"] in (0, 1)
        if not st["from_cache"]:
            assert all(t > 0 for t in st["tune_ms"]) and all(t > 0 for t in st["persist_tune_ms"])
        if design == "persistent":
            assert st["items"] > 0


def test_tuning_cached_per_size_class():
    """A second batch of the same size class takes the first one's tuning."""
    graphs = small_batch()
    with efgpu.Batch(graphs) as b:
        b.autotune("fp64")
        st1 = b.stats()
    with efgpu.Batch(graphs) as b:
        b.autotune("fp64")
        st2 = b.stats()
        ef, D, N = b.compute(prec="fp64")
    assert st2["from_cache"] == 1 and st2["size_class"] == st1["size_class"]
    for k in ("design", "tuned_choice", "persist_choice", "thr8", "thr16", "thr32"):
        assert st2[k] == st1[k], k
    rp, ci = graphs[3]
    oN, oD, oE = oracle.ef(rp, ci)
    sl = slice(int(b.node_off[3]), int(b.node_off[4]))
    assert np.array_equal(N[sl], oN) and np.array_equal(D[sl], oD)


@pytest.mark.parametrize("design", ["phased", "persistent"])
@pytest.mark.parametrize("prec", ["fp32c", "fp64"])
def test_config4_batch512_full_size_sampled(prec, design):
    """The full 512-graph batch (half Watts-Strogatz, half erased configuration
    model with power-law degrees, n ~ U[1e3, 1e5]; 25.5M nodes). On every
    node: N against its closed form, the sum rule sum N = 4 W, and the
    entropy bounds 0 <= EF <= ln N. Against the oracle: 16 random nodes and
    the three largest-degree nodes of every graph, and every node with more
    than 2^24 event sequences (the FP64-finalised seeds)."""
    graphs = gen.batch_512()
    node_off, rp, ci = efgpu.union_csr(graphs)
    n = rp.size - 1
    deg = np.diff(rp).astype(np.int64)
    with efgpu.Batch(graphs) as b:
        ef, D, N = b.compute(prec=prec, design=design)
        if design == "persistent":
            # the two designs: integers bit for bit, EF within the tolerance
            e1, D1, N1 = b.compute(prec=prec, design="phased")
            assert np.array_equal(D1, D) and np.array_equal(N1, N)
            assert np.all(np.abs(e1 - ef) <= 2 * REL[prec] * np.abs(e1))
    src = np.repeat(np.arange(n), deg)
    A = np.bincount(src, weights=deg[ci], minlength=n).astype(np.int64)
    Nc = deg * deg - 2 * deg + A
    assert np.array_equal(N, Nc)
    assert int(N.sum()) == 4 * int((deg * (deg - 1) // 2).sum())
    ok = N > 1
    assert np.all(ef >= 0) and np.all(ef[~ok] == 0) and not np.any(np.signbit(ef))
    assert np.all(ef[ok] <= np.log(N[ok].astype(np.float64)) * (1 + 1e-6))
    rng = np.random.default_rng(512)
    pick = [np.flatnonzero(N > (1 << 24))]
    for i in range(len(graphs)):
        lo, hi = int(node_off[i]), int(node_off[i + 1])
        pick.append(lo + rng.choice(hi - lo, 16, replace=False))
        pick.append(lo + np.argsort(deg[lo:hi], kind="stable")[-3:])
    seeds = np.unique(np.concatenate(pick)).astype(np.int32)
    assert np.count_nonzero(N[seeds] > (1 << 24)) >= 10
    oN, oD, oE = oracle.ef(rp, ci, seeds=seeds, threads=16)
    assert np.array_equal(N[seeds], oN) and np.array_equal(D[seeds], oD)
    err = np.abs(ef[seeds] - oE)
    bad = np.flatnonzero(err > REL[prec] * np.abs(oE))
    assert bad.size == 0, (prec, seeds[bad[:5]], ef[seeds[bad[:5]]], oE[bad[:5]])
    pos = oE > 0
    sys.stderr.write(f"[batch512] {prec} {design}: {seeds.size} oracle seeds, max rel err "
                     f"{float((err[pos] / oE[pos]).max()):.3e}\n")
