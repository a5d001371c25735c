"""The learned surrogate on the GPU: gradients against the CPU oracle,
features against closed forms, training, save/load, and the top-k with exact
rescoring and fallback (needs an MI355X)."""
import sys

import numpy as np
import pytest

import oracle
from oracle import mlp_ref
from paper_2306_00606_amd import efgpu, gen, surrogate
from tests import efref

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _announce(request):
    sys.stderr.write(f"\n[gpu case] {request.node.nodeid}\n")
    sys.stderr.flush()
    yield


def test_gradients_match_cpu_oracle():
    rs = np.random.default_rng(5)
    s = efgpu.Surrogate(seed=3)
    p = mlp_ref.init_params(7)
    p["b1"] = rs.normal(0, 0.2, 64)
    p["b2"] = rs.normal(0, 0.2, 64)
    p["b3"] = np.array([0.1])
    s.set_params(mlp_ref.flatten(p).astype(np.float32))
    P32 = s.params()[0].astype(np.float64)     # the parameters as the GPU holds them
    p32 = mlp_ref.unflatten(P32)
    for rows in (32, 77, 300):
        X = rs.normal(0, 1, (rows, 16)).astype(np.float32)
        y = rs.normal(0, 1, rows).astype(np.float32)
        g, loss = s.gradients(X, y)
        rl, rg = mlp_ref.loss_and_grads(p32, X.astype(np.float64), y.astype(np.float64), bf16=True)
        assert abs(loss - rl) <= 2e-3 * max(1.0, rl), (rows, loss, rl)
        ref = mlp_ref.flatten(rg)
        for name, (a, b) in {"W1": (0, 1024), "b1": (1024, 1088), "W2": (1088, 5184),
                             "b2": (5184, 5248), "w3": (5248, 5312), "b3": (5312, 5313)}.items():
            gn, rn = g[a:b].astype(np.float64), ref[a:b]
            err = np.linalg.norm(gn - rn) / max(np.linalg.norm(rn), 1e-12)
            sys.stderr.write(f"[grad] rows={rows} {name} rel err {err:.2e}\n")
            assert err <= 2e-2, (rows, name, err)


def test_features_match_closed_forms():
    rp, ci = gen.erdos_renyi(150, 0.06, 4)
    n = rp.size - 1
    with efgpu.Graph(rp, ci) as g:
        X, lnN = g.features()
    A = efref.dense_adjacency(n, rp, ci)
    k = A.sum(1).astype(np.float64)
    Asum = A @ k
    B = A @ (k * k)
    T = np.diag(A @ A @ A) / 2
    Q = A @ Asum
    N, D = efref.closed_form_ND(n, rp, ci)
    assert np.allclose(X[:, 0], np.log1p(k), rtol=1e-6)
    assert np.allclose(X[:, 1], np.log1p(Asum), rtol=1e-6)
    assert np.allclose(X[:, 2], np.log1p(B), rtol=1e-6)
    assert np.allclose(X[:, 3], np.log1p(T), rtol=1e-6)
    cc = np.where(k >= 2, 2 * T / np.maximum(k * (k - 1), 1), 0)
    assert np.allclose(X[:, 4], cc, rtol=1e-6, atol=1e-7)
    assert np.allclose(X[:, 6], np.log1p(N), rtol=1e-6)
    assert np.allclose(X[:, 7], np.log1p(D), rtol=1e-6)
    assert np.allclose(X[:, 13], np.log1p(Q), rtol=1e-6)
    ok = N > 0
    assert np.allclose(lnN[ok], np.log(N[ok]), rtol=1e-6)


def test_training_reduces_loss_and_ranks_well():
    graphs = surrogate.training_graphs(seed=1, count=9, small=True)
    X, y = surrogate.labelled_rows(graphs)
    s = efgpu.Surrogate(seed=0)
    P0 = s.params()[0]
    g0, loss0 = s.gradients((X[:4096] - X.mean(0)) / (X.std(0) + 1e-6), y[:4096])
    rep = s.train(X, y, lr=3e-3, epochs=25, batch=2048, seed=2, val_fraction=0.1, patience=5)
    sys.stderr.write(f"[train] {rep}\n")
    assert rep["epochs_run"] >= 1 and rep["train_loss"] < loss0
    assert not np.array_equal(P0, s.params()[0])
    rp, ci = gen.barabasi_albert(20000, 8, 99)
    with efgpu.Graph(rp, ci) as g:
        res = surrogate.evaluate(s, g)
    sys.stderr.write(f"[eval] {res}\n")
    assert res["surrogate"]["spearman"] >= 0.98
    assert res["surrogate"]["spearman"] >= res["degree"]["spearman"]


def test_save_load_roundtrip(tmp_path):
    s = efgpu.Surrogate(seed=11)
    X = np.random.default_rng(0).normal(0, 1, (512, 16)).astype(np.float32)
    y = np.random.default_rng(1).normal(0, 1, 512).astype(np.float32)
    s.train(X, y, epochs=2, batch=128, val_fraction=0.0)
    path = tmp_path / "s.bin"
    s.save(path)
    t = efgpu.Surrogate(seed=99)
    t.load(path)
    for a, b in zip(s.params(), t.params()):
        assert np.array_equal(a, b)


def test_topk_surrogate_rescoring_and_fallback():
    graphs = surrogate.training_graphs(seed=4, count=6, small=True)
    X, y = surrogate.labelled_rows(graphs)
    s = efgpu.Surrogate(seed=0)
    s.train(X, y, epochs=15, batch=2048, val_fraction=0.1)
    rp, ci = gen.barabasi_albert(8000, 5, 17)
    oN, oD, oE = oracle.ef(rp, ci, threads=8)
    with efgpu.Graph(rp, ci) as g:
        k = 50
        nodes, ef, rep = s.topk(g, k, rerank_factor=4, judge_sample=2000, min_spearman=0.0)
        assert rep["fallback"] == 0 and rep["candidates"] == 4 * k
        # rescored values are exact
        assert np.all(np.abs(ef - oE[nodes]) <= 1e-5 * oE[nodes])
        assert np.all(np.diff(ef) <= 0)
        # forced fallback: exact top-k of the whole graph
        nodes2, ef2, rep2 = s.topk(g, k, judge_sample=500, min_spearman=1.5)
        assert rep2["fallback"] == 1
        exact_nodes, exact_ef = g.topk(k)
        assert np.array_equal(nodes2, exact_nodes)
