"""CPU oracle for the surrogate MLP: forward pass, mean-squared-error loss and
its gradients, written out by hand in float64 with NumPy (no autograd).

TEST INFRASTRUCTURE ONLY (imported by tests/ and never by the GPU library).

Network: x (16) -> z1 = x W1 + b1 -> h1 = gelu(z1) (64) -> z2 = h1 W2 + b2 ->
h2 = gelu(z2) (64) -> y = h2 w3 + b3 (1), with the tanh form of GELU
(Hendrycks and Gimpel, "Gaussian Error Linear Units", 2016):
gelu(z) = z/2 (1 + tanh(sqrt(2/pi) (z + 0.044715 z^3))).
Loss L = mean_i (y_i - t_i)^2.

With bf16=True the operands that the GPU kernels round to bfloat16 (x, the
weights W1, W2, w3, the activations h1, h2 fed to the next layer, and in the
backward pass the pre-activation gradients dz2, dz1 fed to the weight and
input gradient products) are rounded the same way (round to nearest even),
and everything else stays in float64; this removes the rounding of the
operands from the comparison and leaves only the accumulation order.
"""
from __future__ import annotations

import math

import numpy as np

F, H = 16, 64


def bf16_round(a):
    """Round float values to the nearest bfloat16 (ties to even), as float64."""
    a32 = np.asarray(a, dtype=np.float32)
    u = a32.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


_C = math.sqrt(2.0 / math.pi)
_A = 0.044715


def gelu(z):
    return 0.5 * z * (1.0 + np.tanh(_C * (z + _A * z * z * z)))


def gelu_grad(z):
    t = np.tanh(_C * (z + _A * z * z * z))
    return 0.5 * (1.0 + t) + 0.5 * z * (1.0 - t * t) * _C * (1.0 + 3.0 * _A * z * z)


def flatten(p):
    """The flat parameter order of the library: W1, b1, W2, b2, w3, b3."""
    return np.concatenate([p["W1"].reshape(-1), p["b1"], p["W2"].reshape(-1), p["b2"],
                           p["w3"], p["b3"]])


def unflatten(v):
    v = np.asarray(v, np.float64)
    return {"W1": v[0:1024].reshape(F, H), "b1": v[1024:1088],
            "W2": v[1088:5184].reshape(H, H), "b2": v[5184:5248], "w3": v[5248:5312],
            "b3": v[5312:5313]}


def init_params(seed: int = 0):
    rs = np.random.default_rng(seed)
    return {
        "W1": rs.normal(0, 1 / math.sqrt(F), (F, H)),
        "b1": np.zeros(H),
        "W2": rs.normal(0, 1 / math.sqrt(H), (H, H)),
        "b2": np.zeros(H),
        "w3": rs.normal(0, 1 / math.sqrt(H), H),
        "b3": np.zeros(1),
    }


def forward(p, X, bf16=False):
    rnd = bf16_round if bf16 else (lambda a: np.asarray(a, np.float64))
    x = rnd(X)
    W1, W2, w3 = rnd(p["W1"]), rnd(p["W2"]), rnd(p["w3"])
    z1 = x @ W1 + p["b1"]
    h1 = rnd(gelu(z1))
    z2 = h1 @ W2 + p["b2"]
    h2 = rnd(gelu(z2))
    y = h2 @ w3 + p["b3"][0]
    return y, {"x": x, "W1": W1, "W2": W2, "w3": w3, "z1": z1, "h1": h1, "z2": z2, "h2": h2}


def loss_and_grads(p, X, t, bf16=False):
    """Returns (loss, grads) with grads holding dL/d(each parameter)."""
    y, c = forward(p, X, bf16)
    n = X.shape[0]
    r = y - t
    loss = float(np.mean(r * r))
    dy = 2.0 * r / n
    g = {}
    g["w3"] = c["h2"].T @ dy
    g["b3"] = np.array([dy.sum()])
    rnd = bf16_round if bf16 else (lambda a: a)
    dh2 = np.outer(dy, c["w3"])
    dz2 = dh2 * gelu_grad(c["z2"])
    g["b2"] = dz2.sum(0)
    dz2 = rnd(dz2)
    g["W2"] = c["h1"].T @ dz2
    dh1 = dz2 @ c["W2"].T
    dz1 = dh1 * gelu_grad(c["z1"])
    g["b1"] = dz1.sum(0)
    dz1 = rnd(dz1)
    g["W1"] = c["x"].T @ dz1
    return loss, g


def spearman(a, b):
    """Spearman rank correlation with average ranks for ties."""
    def ranks(v):
        v = np.asarray(v, np.float64)
        order = np.argsort(v, kind="mergesort")
        r = np.empty(v.size, np.float64)
        sv = v[order]
        i = 0
        while i < v.size:
            j = i
            while j + 1 < v.size and sv[j + 1] == sv[i]:
                j += 1
            r[order[i:j + 1]] = 0.5 * (i + j)
            i = j + 1
        return r
    ra, rb = ranks(a), ranks(b)
    ra -= ra.mean()
    rb -= rb.mean()
    return float((ra * rb).sum() / math.sqrt((ra * ra).sum() * (rb * rb).sum()))
