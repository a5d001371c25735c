"""Top-k selection on the device (needs an MI355X).

The k largest values, ties by node id ascending, is a unique answer: the
library's ranking is compared bit for bit with a plain sort of the same values
(numpy lexsort on (-value, id)), on crafted value arrays with many ties, zeros
and ragged sizes, for k on both sides of the one-workgroup sort limit (4096),
and through ef_topk on graphs whose EF values are all equal.
"""
import sys

import numpy as np
import pytest

from paper_2306_00606_amd import efgpu, gen

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _announce(request):
    sys.stderr.write(f"\n[gpu case] {request.node.nodeid}\n")
    sys.stderr.flush()
    yield


def reference_topk(v, k):
    key = np.where(v > 0, v, 0.0)
    order = np.lexsort((np.arange(v.size), -key))
    return order[:k].astype(np.int32), key[order[:k]]


def values(n, seed):
    """Non-negative doubles with heavy ties: a few distinct levels, exact
    zeros, tiny denormals, and a continuous part."""
    rs = np.random.default_rng(seed)
    v = rs.random(n) * 20.0
    pick = rs.random(n)
    v[pick < 0.3] = rs.choice([1.5, 2.0, 7.25], size=int((pick < 0.3).sum()))
    v[pick > 0.9] = 0.0
    v[(pick > 0.85) & (pick <= 0.9)] = 5e-324
    return v


@pytest.mark.parametrize("n", [1, 2, 63, 1001, 4097, 100000])
def test_topk_values_against_sort(n):
    torch = pytest.importorskip("torch")
    v = values(n, n)
    ks = sorted({k for k in (1, 2, 7, 1000, 4095, 4096, 4097, 50000, n - 1, n) if 1 <= k <= n})
    rp = np.zeros(n + 1, np.int32)
    with efgpu.Graph(rp, np.zeros(0, np.int32)) as g:
        dv = torch.from_numpy(v).cuda()
        for k in ks:
            nodes, ef = g.topk_values(dv, k)
            want_n, want_v = reference_topk(v, k)
            assert np.array_equal(nodes, want_n), (n, k, np.flatnonzero(nodes != want_n)[:5])
            assert np.array_equal(ef.view(np.int64), want_v.view(np.int64)), (n, k)
        # device outputs, twice in a row on the same handle
        for k in ks[-2:]:
            on = torch.empty(k, dtype=torch.int32, device="cuda")
            ov = torch.empty(k, dtype=torch.float64, device="cuda")
            g.topk_values(dv, k, out=(on, ov))
            torch.cuda.synchronize()
            want_n, want_v = reference_topk(v, k)
            assert np.array_equal(on.cpu().numpy(), want_n)
            assert np.array_equal(ov.cpu().numpy(), want_v)


def test_topk_values_all_equal_and_all_zero():
    torch = pytest.importorskip("torch")
    n = 20000
    rp = np.zeros(n + 1, np.int32)
    with efgpu.Graph(rp, np.zeros(0, np.int32)) as g:
        for fill in (3.0, 0.0):
            dv = torch.full((n,), fill, dtype=torch.float64, device="cuda")
            for k in (1, 4096, 4097, n):
                nodes, ef = g.topk_values(dv, k)
                assert np.array_equal(nodes, np.arange(k, dtype=np.int32))
                assert np.all(ef == fill) and not np.any(np.signbit(ef))
        with pytest.raises(efgpu.EFError):
            g.topk_values(dv, n + 1)


@pytest.mark.parametrize("k", [1, 100, 4096, 5000, 10000])
def test_topk_cycle_graph_ties(k):
    """Every node of a cycle has EF = ln 4: the top-k are nodes 0..k-1."""
    n = 10000
    src = np.arange(n, dtype=np.int32)
    rp, ci = gen.from_edges(n, src, (src + 1) % n)
    with efgpu.Graph(rp, ci) as g:
        for prec in ("fp64", "fp32c"):
            nodes, ef = g.topk(k, prec=prec)
            assert np.array_equal(nodes, np.arange(k, dtype=np.int32)), prec
            assert np.allclose(ef, np.log(4.0), rtol=1e-6)
