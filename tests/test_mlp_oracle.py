"""Pins of the FP64 reference network: analytic gradients against central
finite differences, softmax cross-entropy against its definition on a
hand-computable case, and BF16 rounding against the bit-level definition."""
import numpy as np

import oracle.mlp as M


def _params(seed=0):
    rng = np.random.default_rng(seed)
    p = {"mu": rng.normal(size=16) * 0.1, "inv_sigma": 1.0 + rng.random(16)}
    p["W1"] = rng.normal(size=(16, 64)) * 0.3
    p["b1"] = rng.normal(size=64) * 0.1
    p["W2"] = rng.normal(size=(64, 64)) * 0.15
    p["b2"] = rng.normal(size=64) * 0.1
    p["W3"] = rng.normal(size=(64, 4)) * 0.2
    p["b3"] = rng.normal(size=4) * 0.1
    return p


def test_gradients_match_finite_differences():
    rng = np.random.default_rng(1)
    p = _params()
    X = rng.normal(size=(37, 16))
    y = rng.integers(0, 4, size=37)
    cw = np.array([1.0, 2.0, 3.0, 0.5])
    _, g = M.loss_and_grads(p, X, y, cw)
    eps = 1e-6
    for name in ("W1", "b1", "W2", "b2", "W3", "b3"):
        flat = p[name].reshape(-1)
        idx = rng.choice(flat.size, size=min(12, flat.size), replace=False)
        for k in idx:
            old = flat[k]
            flat[k] = old + eps
            lp, _ = M.loss_and_grads(p, X, y, cw)
            flat[k] = old - eps
            lm, _ = M.loss_and_grads(p, X, y, cw)
            flat[k] = old
            fd = (lp - lm) / (2 * eps)
            assert abs(fd - g[name].reshape(-1)[k]) <= 1e-6 * max(1.0, abs(fd)), (name, k)


def test_cross_entropy_definition():
    # zero weights except a diagonal W3 that copies the first 4 hidden units
    p = {k: np.zeros(s) for k, s in M.SIZES}
    p["inv_sigma"][:] = 1.0
    p["b3"] = np.log(np.array([1.0, 2.0, 3.0, 4.0]))
    X = np.zeros((2, 16))
    loss, _ = M.loss_and_grads(p, X, np.array([3, 0]), np.ones(4))
    assert abs(loss - 0.5 * (-np.log(0.4) - np.log(0.1))) < 1e-14


def test_bf16_rounding_and_pack():
    v = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -9, -2.5, 3.0e38, 1e-40])
    r = M.bf16_round(v)
    assert r[0] == 1.0 and r[1] == 1.0  # tie to even
    assert r[2] == 1.0 + 2 ** -7
    assert r[3] == -2.5
    p = _params(3)
    q = M.unpack(M.pack(p))
    assert all(np.array_equal(p[k], q[k]) for k in p)
    assert M.BLOB_LEN == 5540


def test_decision_rule_ties_and_fallback():
    p = {k: np.zeros(s) for k, s in M.SIZES}
    p["inv_sigma"][:] = 1.0
    X = np.zeros((3, 16))
    # all logits equal: tie -> most expensive rule (3); confidence 0.25
    assert list(M.decide(p, X, fallback=[1, 1, 1], conf_min=0.0)) == [3, 3, 3]
    assert list(M.decide(p, X, fallback=[1, 2, 0], conf_min=0.5)) == [1, 2, 0]
