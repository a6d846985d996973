"""FP64 CPU reference of the rule-selector network (test infrastructure only).

16 -> 64 -> 64 -> 4 with ReLU, features standardised as (x - mu) * inv_sigma,
class-weighted softmax cross-entropy:
    z1 = xs W1 + b1, a1 = relu(z1), z2 = a1 W2 + b2, a2 = relu(z2),
    z3 = a2 W3 + b3, p = softmax(z3),
    loss = sum_i c[y_i] (-log p[i, y_i]) / sum_i c[y_i].
Backward pass written out from the chain rule (no autodiff); pinned by
central finite differences in the tests.

forward_bf16 / decide_bf16 take the decision in the precision of a BF16
inference (the selector's own precision): the standardised inputs and the
two hidden activations are rounded to bfloat16 there, products and sums
are exact here (FP64); decide_bf16 also flags the rows whose outcome a
rounding difference in those sums could change.

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


def _ordinal(z, fallback, conf_min):
    """Cheapest class r in (0, 1, 2) whose softmax mass p_0 + ... + p_r is
    at least conf_min (classes ordered by cost); rows where none is keep
    the fallback."""
    e = np.exp(z - z.max(axis=1, keepdims=True))
    C = np.cumsum(e / e.sum(axis=1, keepdims=True), axis=1)
    rule = np.array(np.broadcast_to(np.asarray(fallback), (z.shape[0],)), dtype=np.int64)
    for r in (2, 1, 0):
        rule = np.where(C[:, r] >= conf_min, r, rule)
    return rule, C


def decide(p, X, fallback, conf_min):
    """Rule per row: the cheapest Gauss rule r whose predicted probability of
    meeting the error budget, P(label <= r), is at least conf_min; rows
    where no Gauss rule is keep the fallback."""
    return _ordinal(forward(p, X)["z3"], fallback, conf_min)[0]


def forward_bf16(p, X):
    """Logits with the rounding points of a BF16 inference."""
    xs = bf16_round((np.asarray(X, dtype=np.float64) - p["mu"]) * p["inv_sigma"])
    a1 = bf16_round(np.maximum(xs @ p["W1"] + p["b1"], 0.0))
    a2 = bf16_round(np.maximum(a1 @ p["W2"] + p["b2"], 0.0))
    return a2 @ p["W3"] + p["b3"]


def decide_bf16(p, X, fallback, conf_min, margin=0.01):
    """decide() with forward_bf16.  Returns (rule [P], alternatives [P, 3]):
    the other rules (-1 = none) that a rounding difference in the network's
    sums could give.  The decision only moves when a cumulative probability
    crosses conf_min, and it is monotone in them, so the possible outcomes
    are the classes between the decisions taken at conf_min - margin and at
    conf_min + margin ("no Gauss rule" counted as class 3, the fallback)."""
    z = forward_bf16(p, X)
    P = z.shape[0]
    fb = np.broadcast_to(np.asarray(fallback), (P,))
    none = np.full(P, 3)
    rule3, C = _ordinal(z, none, conf_min)
    lo, _ = _ordinal(z, none, conf_min - margin)
    hi, _ = _ordinal(z, none, conf_min + margin)
    rule = np.where(rule3 == 3, fb, rule3)
    alt = np.full((P, 3), -1, dtype=np.int64)
    for row in np.nonzero(lo != hi)[0]:
        outs = [r if r < 3 else int(fb[row]) for r in range(lo[row], hi[row] + 1)]
        outs = [o for o in outs if o != rule[row]][:3]
        alt[row, :len(outs)] = outs
    return rule, alt
