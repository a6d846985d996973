"""FP64 CPU reference of the rule-selector network (test infrastructure only).

16 -> 64 -> 64 -> 4 with ReLU, features standardised as (x - mu) * inv_sigma,
class-weighted softmax cross-entropy:
    z1 = xs W1 + b1, a1 = relu(z1), z2 = a1 W2 + b2, a2 = relu(z2),
    z3 = a2 W3 + b3, p = softmax(z3),
    loss = sum_i c[y_i] (-log p[i, y_i]) / sum_i c[y_i].
Backward pass written out from the chain rule (no autodiff); pinned by
central finite differences in the tests.

Parameter blob layout (the same order as the library's packed BF16 blob):
mu[16], inv_sigma[16], W1[16][64], b1[64], W2[64][64], b2[64], W3[64][4], b3[4].
"""
from __future__ import annotations

import numpy as np

SIZES = [("mu", (16,)), ("inv_sigma", (16,)), ("W1", (16, 64)), ("b1", (64,)), ("W2", (64, 64)), ("b2", (64,)),
         ("W3", (64, 4)), ("b3", (4,))]
BLOB_LEN = sum(int(np.prod(s)) for _, s in SIZES)


def unpack(blob):
    blob = np.asarray(blob, dtype=np.float64)
    assert blob.size == BLOB_LEN, blob.size
    out, o = {}, 0
    for name, shp in SIZES:
        n = int(np.prod(shp))
        out[name] = blob[o:o + n].reshape(shp)
        o += n
    return out


def pack(p):
    return np.concatenate([np.asarray(p[name], dtype=np.float64).ravel() for name, _ in SIZES])


def bf16_round(a):
    """Round float64 values to the nearest bfloat16 (ties to even) and back."""
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    u = (u + 0x7FFF + lsb) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def forward(p, X):
    xs = (np.asarray(X, dtype=np.float64) - p["mu"]) * p["inv_sigma"]
    z1 = xs @ p["W1"] + p["b1"]
    a1 = np.maximum(z1, 0.0)
    z2 = a1 @ p["W2"] + p["b2"]
    a2 = np.maximum(z2, 0.0)
    z3 = a2 @ p["W3"] + p["b3"]
    return dict(xs=xs, z1=z1, a1=a1, z2=z2, a2=a2, z3=z3)


def loss_and_grads(p, X, y, class_w):
    """Weighted cross-entropy and its gradients w.r.t. W1, b1, W2, b2, W3, b3
    (mu and inv_sigma are fixed: zero gradient)."""
    f = forward(p, X)
    z3 = f["z3"]
    zmax = z3.max(axis=1, keepdims=True)
    e = np.exp(z3 - zmax)
    prob = e / e.sum(axis=1, keepdims=True)
    y = np.asarray(y, dtype=np.int64)
    w = np.asarray(class_w, dtype=np.float64)[y]
    W = w.sum()
    loss = float(np.sum(w * -np.log(prob[np.arange(y.size), y])) / W)
    d3 = prob.copy()
    d3[np.arange(y.size), y] -= 1.0
    d3 *= (w / W)[:, None]
    g = {"mu": np.zeros(16), "inv_sigma": np.zeros(16)}
    g["W3"] = f["a2"].T @ d3
    g["b3"] = d3.sum(axis=0)
    d2 = (d3 @ p["W3"].T) * (f["z2"] > 0)
    g["W2"] = f["a1"].T @ d2
    g["b2"] = d2.sum(axis=0)
    d1 = (d2 @ p["W2"].T) * (f["z1"] > 0)
    g["W1"] = f["xs"].T @ d1
    g["b1"] = d1.sum(axis=0)
    return loss, g


def decide(p, X, fallback, conf_min):
    """Rule per row: argmax of the logits (ties to the more expensive rule,
    i.e. the larger index); rows whose softmax maximum is below conf_min
    keep the fallback rule."""
    z3 = forward(p, X)["z3"]
    zmax = z3.max(axis=1, keepdims=True)
    e = np.exp(z3 - zmax)
    prob = e / e.sum(axis=1, keepdims=True)
    arg = 3 - np.argmax(z3[:, ::-1], axis=1)
    keep = prob.max(axis=1) < conf_min
    return np.where(keep, np.asarray(fallback), arg)
