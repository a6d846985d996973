"""Writes selector_blob.json: a rule-selector network trained on the CPU
from labels the oracle computes (the input of the learned-policy parity
and gain tests; no value in it comes from the library).

Pairs: for seeded random nodes of two meshes (the Gaussian-swirl box at
10^3 cells and the vortex-ring box at 32 x 32 x 11 cells), every tet whose
fixed-rule pair is ray traced and does not contain the node (the pairs the
selector decides).  Label: the cheapest Gauss rule (G1 < G4 < G11) whose
relative error against the cone-decomposition reference of the pair is at
most TAU, else ray tracing.  Features: oracle.features.  Network: the
16-64-64-4 selector trained with Adam on the FP64 loss and gradients of
oracle.mlp (class-weighted cross-entropy), then rounded to bfloat16.

    python tests/golden/make_selector_blob.py
"""
from __future__ import annotations

import json
import os
import sys
from multiprocessing import Pool

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workloads as W  # noqa: E402
from oracle import features as F  # noqa: E402
from oracle import mlp as MLP  # noqa: E402
from oracle import references as R  # noqa: E402

TAU = 0.01
SEED = 4
REF_ORDER = 20


def candidate_pairs(mesh, n_nodes, rng):
    tg = np.sort(rng.choice(mesh.n_nodes, n_nodes, replace=False))
    _, rules = oracle.evaluate(mesh.xyz, mesh.omega, mesh.tets, oracle.make_policy("fixed"), targets=tg,
                               return_rules=True)
    out = []
    for k, i in enumerate(tg):
        ts = np.nonzero(rules[k] == 3)[0]
        ts = ts[~np.any(mesh.tets[ts] == i, axis=1)]
        out += [(int(i), int(t)) for t in ts]
    return np.array(out, dtype=np.int64)


def _label(args):
    x, tv, tw = args
    ref = R.tet_cone_brute_force(x, tv, tw, order=REF_ORDER)
    n = np.linalg.norm(ref)
    errs = [np.linalg.norm(oracle.pair(x, tv, tw, r) - ref) / n for r in range(3)]
    return next((r for r in range(3) if errs[r] <= TAU), 3)


def dataset(mesh, n_nodes, rng, pool):
    pairs = candidate_pairs(mesh, n_nodes, rng)
    hb = oracle.mean_edge(mesh.xyz, mesh.tets)
    X = F.pair_features_batch(mesh.xyz[pairs[:, 0]], mesh.xyz[mesh.tets[pairs[:, 1]]], hb,
                              np.zeros(len(pairs), bool))
    args = [(mesh.xyz[i], mesh.xyz[mesh.tets[t]], mesh.omega[mesh.tets[t]]) for i, t in pairs]
    y = np.array(pool.map(_label, args, chunksize=64), dtype=np.int64)
    return X, y


def train(X, y, rng, epochs=60, batch=512, lr=2e-3):
    mu = MLP.bf16_round(X.mean(axis=0))
    sd = X.std(axis=0)
    isg = MLP.bf16_round(np.where(sd > 1e-12, 1.0 / np.maximum(sd, 1e-12), 0.0))
    p = {"mu": mu, "inv_sigma": isg,
         "W1": rng.normal(size=(16, 64)) * np.sqrt(2 / 16), "b1": np.zeros(64),
         "W2": rng.normal(size=(64, 64)) * np.sqrt(2 / 64), "b2": np.zeros(64),
         "W3": rng.normal(size=(64, 4)) * np.sqrt(1 / 64), "b3": np.zeros(4)}
    cnt = np.bincount(y, minlength=4).astype(np.float64)
    cw = np.where(cnt > 0, 1.0 / np.sqrt(np.maximum(cnt, 1.0)), 0.0)
    cw /= cw.max()
    names = ["W1", "b1", "W2", "b2", "W3", "b3"]
    m1 = {k: np.zeros_like(p[k]) for k in names}
    m2 = {k: np.zeros_like(p[k]) for k in names}
    step = 0
    for ep in range(epochs):
        order = rng.permutation(len(y))
        for s in range(0, len(y), batch):
            idx = order[s:s + batch]
            _, g = MLP.loss_and_grads(p, X[idx], y[idx], cw)
            step += 1
            for k in names:
                m1[k] = 0.9 * m1[k] + 0.1 * g[k]
                m2[k] = 0.999 * m2[k] + 0.001 * g[k] ** 2
                p[k] = p[k] - lr * (m1[k] / (1 - 0.9 ** step)) / (np.sqrt(m2[k] / (1 - 0.999 ** step)) + 1e-8)
    return p, cw


def main():
    rng = np.random.default_rng(SEED)
    meshes = [(W.make_config("C1"), 400), (W.make_config("C2", scale=(32, 32, 11)), 200)]
    Xs, ys = [], []
    with Pool(min(8, os.cpu_count() or 1)) as pool:
        for mesh, k in meshes:
            X, y = dataset(mesh, k, rng, pool)
            Xs.append(X)
            ys.append(y)
            print(f"{mesh.name}: {len(y)} pairs, labels {np.bincount(y, minlength=4).tolist()}", flush=True)
    X, y = np.concatenate(Xs), np.concatenate(ys)
    perm = rng.permutation(len(y))
    nval = len(y) // 10
    va, tr = perm[:nval], perm[nval:]
    p, cw = train(X[tr], y[tr], rng)
    flat = MLP.bf16_round(MLP.pack(p))
    q = MLP.unpack(flat)
    acc = float(np.mean(np.argmax(MLP.forward_bf16(q, X[va]), axis=1) == y[va]))
    bits = (flat.astype(np.float32).view(np.uint32) >> 16).astype(np.uint16)
    out = {"description": "rule selector trained on oracle labels (pairs the fixed rule ray traces, not incident)",
           "tau": TAU, "seed": SEED, "reference_order": REF_ORDER, "n_pairs": int(len(y)),
           "label_counts": np.bincount(y, minlength=4).tolist(), "class_weights": cw.tolist(),
           "val_accuracy": acc, "conf_min": 0.9, "val_majority": float(np.max(np.bincount(y[va], minlength=4)) / len(va)),
           "blob_bf16_bits": bits.tolist()}
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "selector_blob.json")
    with open(path, "w") as f:
        json.dump(out, f)
    print(f"validation accuracy {acc:.3f} (majority {out['val_majority']:.3f}); wrote {path}")


if __name__ == "__main__":
    main()
