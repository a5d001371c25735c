"""Batched computation (disjoint union, captured HIP graph, tuned thresholds)
against the oracle and against one-graph-at-a-time computation (needs an
MI355X)."""
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


@pytest.mark.parametrize("prec", ["fp32c", "fp64"])
def test_batch_matches_oracle_and_single_graphs(prec):
    graphs = small_batch()
    with efgpu.Batch(graphs, validate=True) as b:
        ef, D, N = b.compute(prec=prec)
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


def test_graph_replays_match_eager():
    """Replay the captured graph several times, with unrelated eager work and
    synchronisations in between; every replay must equal the first result
    bit for bit."""
    torch = pytest.importorskip("torch")
    graphs = small_batch()
    other = gen.rmat(11, 8, 3, perm_seed=4)
    with efgpu.Batch(graphs) as b, efgpu.Graph(*other) as g:
        ref = b.compute(prec="fp32c")
        dev = torch.device("cuda:0")
        ef_t = torch.empty(b.n, dtype=torch.float64, device=dev)
        D_t = torch.empty(b.n, dtype=torch.int64, device=dev)
        N_t = torch.empty(b.n, dtype=torch.int64, device=dev)
        for r in range(5):
            g.compute(algo="per_seed", prec="fp64")  # eager work on the same device
            torch.cuda.synchronize()
            ef_t.fill_(-1.0)
            b.compute(prec="fp32c", out=(ef_t, D_t, N_t), profile=(r == 4))
            torch.cuda.synchronize()
            assert np.array_equal(ef_t.cpu().numpy().view(np.int64), ref[0].view(np.int64)), r
            assert np.array_equal(D_t.cpu().numpy(), ref[1])
            assert np.array_equal(N_t.cpu().numpy(), ref[2])
        st = b.stats()
        assert st["replay_ms"] > 0
        assert 0 <= st["tuned_choice"] < 8
        assert all(t > 0 for t in st["tune_ms"])
