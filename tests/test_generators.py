"""The seeded generators: determinism and simple-graph output (no GPU)."""
import numpy as np
import pytest

from paper_2306_00606_amd import gen


def check_simple_csr(rp, ci):
    n = rp.size - 1
    assert rp[0] == 0 and np.all(np.diff(rp) >= 0) and rp[-1] == ci.size
    assert ci.size == 0 or (ci.min() >= 0 and ci.max() < n)
    src = np.repeat(np.arange(n), np.diff(rp))
    assert not np.any(src == ci), "self-loop"
    for i in range(n):
        row = ci[rp[i]:rp[i + 1]]
        assert np.all(np.diff(row) > 0), "unsorted or duplicate"
    fwd = set(zip(src.tolist(), ci.tolist()))
    assert all((v, u) in fwd for (u, v) in fwd), "not symmetric"


GENS = [
    ("er", lambda s: gen.erdos_renyi(300, 0.03, s)),
    ("ba", lambda s: gen.barabasi_albert(400, 3, s)),
    ("rmat", lambda s: gen.rmat(9, 8, s, perm_seed=s + 1)),
    ("ws", lambda s: gen.watts_strogatz(300, 6, 0.2, s)),
    ("cm", lambda s: gen.config_model(300, 2.3, s)),
]


@pytest.mark.parametrize("name,f", GENS)
def test_deterministic_and_simple(name, f):
    a = f(5)
    b = f(5)
    c = f(6)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    assert not (a[0].size == c[0].size and np.array_equal(a[1], c[1]))
    check_simple_csr(*a)


def test_sizes():
    rp, ci = gen.er_1000(1)
    assert rp.size == 1001 and 6.5 < ci.size / 1000 < 9.5
    rp, ci = gen.barabasi_albert(2000, 5, 2)
    assert ci.size == 2 * (5 + 5 * (2000 - 6))
    rp, ci = gen.rmat(10, 10, 1)
    assert rp.size == 1025 and ci.size <= 2 * 10 * 1024
    rp, ci = gen.watts_strogatz(500, 4, 0.0, 1)
    assert np.all(np.diff(rp) == 4)


def test_from_edges_cleans_input():
    rp, ci = gen.from_edges(4, [0, 1, 1, 2, 3], [1, 0, 1, 3, 2])
    assert rp.tolist() == [0, 1, 2, 3, 4] and ci.tolist() == [1, 0, 3, 2]
    with pytest.raises(ValueError):
        gen.from_edges(2, [0], [5])
