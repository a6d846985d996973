"""Training the learned rule selector on the GPU with the library's kernels.

Pairs: bs_learn_sample_pairs (the pairs the fixed rule ray-traces whose tet
does not contain the node, for seeded random nodes).  Labels:
bs_learn_pairs (the cheapest Gauss rule whose error against a
high-accuracy value of the pair's integral is at most tau, else ray
tracing).  Network: bs_mlp_train (BF16 forward and backward on the matrix
cores, Adam on FP32 master weights), class-weighted by the inverse square
root of the label counts.  The blob it returns is what bs_set_policy takes
for BS_POLICY_LEARNED.

evaluate() measures a trained network on pairs of another mesh (held out):
label accuracy, and the decisions the library takes with it (the cheapest
Gauss rule whose cumulative softmax mass reaches conf_min, else ray
tracing): the share of pairs moved off ray tracing and the share moved to a
rule whose actual error exceeds the budget.
"""
from __future__ import annotations

import time

import numpy as np

from . import (BS_POLICY_FIXED, bs_learn_pairs, bs_learn_sample_pairs, bs_mesh_free, bs_mesh_upload, bs_mlp_logits,
               bs_mlp_train, bs_set_policy)


def _pairs_of(mesh_arrays, max_pairs, tau, seed):
    xyz, omega, tets = mesh_arrays
    h = bs_mesh_upload(xyz, omega, tets)
    try:
        bs_set_policy(h, kind=BS_POLICY_FIXED)
        pairs = bs_learn_sample_pairs(h, max_pairs, seed)
        return bs_learn_pairs(h, pairs, tau)
    finally:
        bs_mesh_free(h)


def train(meshes, tau=0.01, pairs_per_mesh=100_000, epochs=30, batch=1024, lr=2e-3, seed=4, val_frac=0.1,
          pairs_total=None):
    """meshes: iterable of (xyz, omega, tets); pairs_per_mesh: an int, or
    one cap per mesh; with pairs_total the meshes are taken in order, each
    giving as many pairs as it has up to what is left of the total.
    Returns (blob uint16 [5540], info dict: pairs, label counts, validation
    accuracy and majority share, final loss, seconds)."""
    import torch

    t0 = time.perf_counter()
    meshes = list(meshes)
    caps = list(pairs_per_mesh) if hasattr(pairs_per_mesh, "__len__") else [pairs_per_mesh] * len(meshes)
    feats, labels = [], []
    left = pairs_total
    for mesh, cap in zip(meshes, caps):
        if pairs_total is not None:
            cap = left
            if cap <= 0:
                break
        f, y, _ = _pairs_of(mesh, cap, tau, seed)
        feats.append(f)
        labels.append(y)
        if pairs_total is not None:
            left -= int(y.shape[0])
    F = torch.cat(feats)
    Y = torch.cat(labels)
    t_label = time.perf_counter() - t0
    gen = torch.Generator().manual_seed(seed)
    perm = torch.randperm(Y.shape[0], generator=gen).to(F.device)
    F, Y = F[perm].contiguous(), Y[perm].contiguous()
    nval = int(Y.shape[0] * val_frac)
    counts = torch.bincount(Y.long(), minlength=4).cpu().numpy().astype(np.float64)
    cw = np.where(counts > 0, 1.0 / np.sqrt(np.maximum(counts, 1.0)), 0.0)
    cw /= cw.max()
    blob, losses = bs_mlp_train(F[nval:], Y[nval:], epochs=epochs, batch=batch, lr=lr, class_w=tuple(cw), seed=seed)
    z = bs_mlp_logits(blob, F[:nval]).cpu().numpy()
    yv = Y[:nval].cpu().numpy()
    rv, bv = recall(np.argmax(z, axis=1), yv)
    info = {"pairs": int(Y.shape[0]), "pairs_by_mesh": [int(y.shape[0]) for y in labels],
            "label_counts": counts.astype(int).tolist(), "tau": tau, "epochs": epochs, "batch": batch,
            "val_accuracy": float(np.mean(np.argmax(z, axis=1) == yv)),
            "val_recall": rv, "val_balanced_accuracy": bv,
            "val_majority": float(np.max(np.bincount(yv, minlength=4)) / max(1, len(yv))),
            "final_loss": float(losses[-1]) if len(losses) else None, "label_seconds": t_label,
            "seconds": time.perf_counter() - t0}
    return blob, info


def recall(pred, labels):
    """Per-class recall (share of each label's pairs predicted as it, None
    for an absent label) and balanced accuracy (their mean over present
    labels), labels and predictions in 0..3."""
    r = []
    for c in range(4):
        k = labels == c
        r.append(float(np.mean(pred[k] == c)) if np.any(k) else None)
    present = [x for x in r if x is not None]
    return r, float(np.mean(present)) if present else None


def decide(logits, conf_min):
    """The library's decision from logits [n, 4] over (G1, G4, G11, RT): the
    cheapest Gauss rule whose cumulative softmax mass reaches conf_min, else
    ray tracing (3)."""
    z = logits - logits.max(axis=1, keepdims=True)
    e = np.exp(z)
    cum = np.cumsum(e[:, :3], axis=1)
    need = conf_min * e.sum(axis=1)
    rule = np.full(len(z), 3, dtype=np.int64)
    for r in (2, 1, 0):
        rule = np.where(cum[:, r] >= need, r, rule)
    return rule


def evaluate(blob, mesh_arrays, pairs=1_000_000, tau=0.01, conf_min=0.9, seed=9):
    """The network on pairs of one mesh (held out from training): label
    accuracy and majority share; with the library's decision at conf_min,
    the share of pairs moved to a Gauss rule and the share moved to a rule
    whose error (against the pair's high-accuracy value) exceeds tau.  The
    labels are imbalanced (most pairs take the 4-point rule) and training
    weights the classes, so per-class recall and balanced accuracy say more
    than raw accuracy against the majority share."""
    f, y, err = _pairs_of(mesh_arrays, pairs, tau, seed)
    z = bs_mlp_logits(blob, f).cpu().numpy()
    yl = y.cpu().numpy().astype(np.int64)
    e = err.cpu().numpy()
    rule = decide(z, conf_min)
    rc, bal = recall(np.argmax(z, axis=1), yl)
    moved = rule < 3
    unsafe = moved & (e[np.arange(len(rule)), np.minimum(rule, 2)] > tau)
    return {"pairs": int(len(yl)), "accuracy": float(np.mean(np.argmax(z, axis=1) == yl)),
            "recall": rc, "balanced_accuracy": bal,
            "majority": float(np.max(np.bincount(yl, minlength=4)) / max(1, len(yl))),
            "label_counts": np.bincount(yl, minlength=4).tolist(), "conf_min": conf_min,
            "moved": float(np.mean(moved)), "moved_with_error_above_tau": float(np.mean(unsafe)),
            "labels_gauss": float(np.mean(yl < 3))}


# The selector of the learned policy as the library's benchmark and
# Lagrangian run use it: 10 million pairs, all of the swirl box's and the
# rest from the ring box, batches of 4096, eight epochs.
TRAINING = dict(tau=0.01, pairs_total=10_000_000, epochs=8, batch=4096, lr=2e-3, seed=4)


def train_selector(make_config, held_out=("C3",), held_out_pairs=1_000_000):
    """Train on the swirl box (C1) and the ring box (C2) as TRAINING says
    (validation on a tenth of those pairs held back from training), then
    evaluate on pairs of the held-out workloads.  make_config: the workload
    builder (name -> mesh)."""
    train_meshes = [make_config("C1"), make_config("C2")]
    blob, info = train([(t.xyz, t.omega, t.tets) for t in train_meshes], **TRAINING)
    info["trained_on"] = [t.name for t in train_meshes]
    ev = {}
    for name in held_out:
        m = make_config(name)
        ev[name] = evaluate(blob, (m.xyz, m.omega, m.tets), pairs=held_out_pairs, tau=TRAINING["tau"])
    info["held_out"] = ev
    return blob, info
