"""Pins of the surrogate's CPU oracle (``oracle/mlp_ref.py``) against an
independent route: the same network built from torch operations in float64
and differentiated by torch's autograd (CPU). The forward pass, the loss and
all six parameter gradients must agree element by element.

The BF16 mode rounds chosen operands to bfloat16; the torch network rounds
the same operands with torch's own bfloat16 conversion (round to nearest
even), forward values with a straight-through rounding and the two
pre-activation gradients that feed the weight products with a rounding of
the gradient only, so autograd reproduces the same arithmetic by a different
route.

Each planted mistake in a copy of ``mlp_ref`` (a dropped bias, swapped
layers, a wrong GELU derivative, a transposed product, a missing rounding)
must make the comparison fail.
"""
from __future__ import annotations

import importlib.util
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

REF_PATH = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle",
                        "mlp_ref.py")


def _load_ref(src=None):
    spec = importlib.util.spec_from_loader("mlp_ref_copy", loader=None)
    mod = importlib.util.module_from_spec(spec)
    if src is None:
        with open(REF_PATH) as f:
            src = f.read()
    exec(compile(src, REF_PATH, "exec"), mod.__dict__)
    return mod


class _RoundST(torch.autograd.Function):
    """bfloat16 rounding of the value; the gradient passes unchanged."""

    @staticmethod
    def forward(ctx, x):
        return x.to(torch.bfloat16).to(torch.float64)

    @staticmethod
    def backward(ctx, g):
        return g


class _RoundGrad(torch.autograd.Function):
    """Identity on the value; the gradient is rounded to bfloat16."""

    @staticmethod
    def forward(ctx, x):
        return x.clone()

    @staticmethod
    def backward(ctx, g):
        return g.to(torch.bfloat16).to(torch.float64)


def torch_reference(p, X, t, bf16):
    P = {k: torch.tensor(np.asarray(v, np.float64), requires_grad=True) for k, v in p.items()}
    x = torch.tensor(np.asarray(X, np.float64))
    tt = torch.tensor(np.asarray(t, np.float64))
    r = _RoundST.apply if bf16 else (lambda a: a)
    g = _RoundGrad.apply if bf16 else (lambda a: a)
    def gelu(a):  # the tanh form
        return torch.nn.functional.gelu(a, approximate="tanh")
    xr = r(x)
    z1 = g(xr @ r(P["W1"])) + P["b1"]
    h1 = r(gelu(z1))
    z2 = g(h1 @ r(P["W2"])) + P["b2"]
    h2 = r(gelu(z2))
    y = h2 @ r(P["w3"]) + P["b3"][0]
    loss = torch.mean((y - tt) ** 2)
    loss.backward()
    return (y.detach().numpy(), float(loss.detach()),
            {k: v.grad.numpy() for k, v in P.items()})


def _case(seed):
    rs = np.random.default_rng(seed)
    ref = _load_ref()
    p = ref.init_params(seed)
    p["b1"] = rs.normal(0, 0.2, 64)
    p["b2"] = rs.normal(0, 0.2, 64)
    p["b3"] = np.array([0.37])
    X = rs.normal(0, 1.5, (33, 16))
    t = rs.normal(0, 1, 33)
    return p, X, t


def agrees(ref, bf16, seed=3):
    """True when the copy `ref` of the oracle matches torch autograd."""
    p, X, t = _case(seed)
    y_t, loss_t, g_t = torch_reference(p, X, t, bf16)
    y, _ = ref.forward({k: v.copy() for k, v in p.items()}, X, bf16=bf16)
    loss, g = ref.loss_and_grads({k: v.copy() for k, v in p.items()}, X, t, bf16=bf16)
    rel = 1e-12

    def close(a, b):
        a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
        return a.shape == b.shape and np.all(np.abs(a - b) <= rel * np.maximum(1.0, np.abs(b)))
    if not close(y, y_t) or not close(loss, loss_t):
        return False
    return all(close(g[k], g_t[k]) for k in ("W1", "b1", "W2", "b2", "w3", "b3"))


@pytest.mark.parametrize("bf16", [False, True])
@pytest.mark.parametrize("seed", [3, 11])
def test_mlp_oracle_matches_torch_autograd(bf16, seed):
    assert agrees(_load_ref(), bf16, seed)


# (site, replacement) in mlp_ref.py, and the mode in which it must be caught
MLP_MUTANTS = {
    "drop_b2": ("z2 = h1 @ W2 + p[\"b2\"]", "z2 = h1 @ W2", False),
    "swap_layer_weights": ("z2 = h1 @ W2 + p[\"b2\"]", "z2 = h1 @ W2.T + p[\"b2\"]", False),
    "gelu_grad_sign": ("+ 0.5 * z * (1.0 - t * t)", "- 0.5 * z * (1.0 - t * t)", False),
    "grad_W2_transposed": ("g[\"W2\"] = c[\"h1\"].T @ dz2", "g[\"W2\"] = (c[\"h1\"].T @ dz2).T", False),
    "loss_not_mean": ("dy = 2.0 * r / n", "dy = 2.0 * r", False),
    "b1_grad_after_rounding": ("g[\"b1\"] = dz1.sum(0)\n    dz1 = rnd(dz1)",
                               "dz1 = rnd(dz1)\n    g[\"b1\"] = dz1.sum(0)", True),
    "h2_not_rounded": ("h2 = rnd(gelu(z2))", "h2 = gelu(z2)", True),
}


@pytest.mark.parametrize("name", sorted(MLP_MUTANTS))
def test_mlp_planted_mistakes_are_caught(name):
    old, new, bf16 = MLP_MUTANTS[name]
    with open(REF_PATH) as f:
        src = f.read()
    assert src.count(old) == 1, f"mutation site for {name} not found exactly once"
    assert not agrees(_load_ref(src.replace(old, new)), bf16), f"mutant {name} survived"
