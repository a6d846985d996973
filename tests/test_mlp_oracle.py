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


def test_decision_rule_cumulative_and_fallback():
    """All logits equal: p = 1/4 each, so P(label <= r) = (r + 1)/4; the
    cheapest rule reaching conf_min is chosen, else the fallback."""
    p = {k: np.zeros(s) for k, s in M.SIZES}
    p["inv_sigma"][:] = 1.0
    X = np.zeros((3, 16))
    assert list(M.decide(p, X, fallback=[3, 3, 3], conf_min=0.2)) == [0, 0, 0]
    assert list(M.decide(p, X, fallback=[3, 3, 3], conf_min=0.5)) == [1, 1, 1]
    assert list(M.decide(p, X, fallback=[3, 3, 3], conf_min=0.7)) == [2, 2, 2]
    assert list(M.decide(p, X, fallback=[3, 1, 0], conf_min=0.9)) == [3, 1, 0]
    # one logit up: G4 gets e/(e+3) of the mass
    p["b3"][:] = [0.0, 1.0, 0.0, 0.0]
    g4 = np.e / (np.e + 3)
    assert list(M.decide(p, X[:1], fallback=3, conf_min=g4 + 1 / (np.e + 3) - 1e-9)) == [1]
    assert list(M.decide(p, X[:1], fallback=3, conf_min=g4 + 1 / (np.e + 3) + 1e-9)) == [2]
    # the BF16 variant agrees away from the threshold and flags rows near it
    r, alt = M.decide_bf16(p, X[:1], 3, conf_min=g4 + 1 / (np.e + 3) + 1e-3, margin=1e-2)
    assert r[0] == 2 and 1 in alt[0]


def test_pair_features_batch_matches_definition():
    import oracle
    import workloads as W
    from oracle import features as F

    m = W.make_config("C1")
    rng = np.random.default_rng(0)
    tets = rng.integers(0, m.n_tets, 200)
    nodes = np.where(rng.random(200) < 0.3, m.tets[tets, 0], rng.integers(0, m.n_nodes, 200))
    hb = oracle.mean_edge(m.xyz, m.tets)
    inc = np.array([n in m.tets[t] for n, t in zip(nodes, tets)])
    B = F.pair_features_batch(m.xyz[nodes], m.xyz[m.tets[tets]], hb, inc)
    S = np.stack([F.pair_features(m.xyz[n], m.xyz[m.tets[t]], hb, i) for n, t, i in zip(nodes, tets, inc)])
    assert np.allclose(B, S, rtol=1e-12, atol=1e-12)
