"""Top-k without allocation (needs an MI355X).

ef_topk_values_noalloc runs the top-k selection on a fixed device scratch
array; its result must equal ef_topk_values (the same selection on workspace
held by a graph handle) bit for bit, on two calls in a row, the second with a
smaller input, and device memory must not change across a call.
"""
import sys

import numpy as np
import pytest

from paper_2306_00606_amd import efgpu

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _announce(request):
    sys.stderr.write(f"\n[gpu case] {request.node.nodeid}\n")
    sys.stderr.flush()
    yield


def values(n, seed):
    rs = np.random.default_rng(seed)
    v = rs.random(n) * 20.0
    pick = rs.random(n)
    v[pick < 0.3] = rs.choice([1.5, 2.0, 7.25], size=int((pick < 0.3).sum()))
    v[pick > 0.9] = 0.0
    return v


def with_handle(v, k):
    torch = pytest.importorskip("torch")
    with efgpu.Graph(np.zeros(v.size + 1, np.int32), np.zeros(0, np.int32)) as g:
        return g.topk_values(torch.from_numpy(v).cuda(), k)


def test_noalloc_topk_equals_topk_values_twice():
    torch = pytest.importorskip("torch")
    # the library's first kernel launch in a fresh process loads its code
    # objects (and with them the fixed array): not part of the calls checked
    warm = torch.ones(8, dtype=torch.float64, device="cuda")
    efgpu.topk_values_noalloc(warm, 8, torch.empty(8, dtype=torch.int32, device="cuda"))
    torch.cuda.synchronize()
    # first call: LSD sort path (k > 4096); second, smaller: LDS sort path
    for n, k in ((300000, 50000), (30001, 3000), (5, 5)):
        v = values(n, n)
        dv = torch.from_numpy(v).cuda()
        nodes = torch.full((k,), -1, dtype=torch.int32, device="cuda")
        vals = torch.full((k,), -1.0, dtype=torch.float64, device="cuda")
        torch.cuda.synchronize()
        free0 = torch.cuda.mem_get_info()[0]
        efgpu.topk_values_noalloc(dv, k, nodes, vals)
        torch.cuda.synchronize()
        free1 = torch.cuda.mem_get_info()[0]
        want_n, want_v = with_handle(v, k)
        assert np.array_equal(nodes.cpu().numpy(), want_n), (n, k)
        assert np.array_equal(vals.cpu().numpy().view(np.int64), want_v.view(np.int64)), (n, k)
        order = np.lexsort((np.arange(n), -v))[:k]
        assert np.array_equal(want_n, order), (n, k)
        assert free1 == free0, f"device memory changed across the call: {free0} -> {free1}"
    # values output is nullable
    v = values(1000, 3)
    nodes = torch.empty(10, dtype=torch.int32, device="cuda")
    efgpu.topk_values_noalloc(torch.from_numpy(v).cuda(), 10, nodes, None)
    torch.cuda.synchronize()
    assert np.array_equal(nodes.cpu().numpy(), np.lexsort((np.arange(1000), -v))[:10])


def test_noalloc_topk_rejects_bad_sizes():
    torch = pytest.importorskip("torch")
    L = efgpu.lib()
    dv = torch.zeros(70000, dtype=torch.float64, device="cuda")
    nodes = torch.empty(70000, dtype=torch.int32, device="cuda")
    for n, k, flags in ((70000, 65537, efgpu.EF_OUT_DEVICE), (10, 11, efgpu.EF_OUT_DEVICE),
                        (10, 5, 0), (-1, 0, efgpu.EF_OUT_DEVICE)):
        st = L.ef_topk_values_noalloc(dv.data_ptr(), n, k, nodes.data_ptr(), None, flags, None)
        assert efgpu.STATUS_NAMES[st] == "EF_ERR_ARG", (n, k, flags)
    # the largest accepted size works
    v = values(70000, 9)
    dv = torch.from_numpy(v).cuda()
    efgpu.topk_values_noalloc(dv, 65536, nodes)
    torch.cuda.synchronize()
    assert np.array_equal(nodes[:65536].cpu().numpy(), np.lexsort((np.arange(70000), -v))[:65536])
