"""Training the learned rule selector on the GPU with the library's kernels.

Pairs: bs_learn_sample_pairs (the pairs the fixed rule ray-traces whose tet
does not contain the node, for seeded random nodes).  Labels:
bs_learn_pairs (the cheapest Gauss rule whose error against a
high-accuracy value of the pair's integral is at most tau, else ray
tracing).  Network: bs_mlp_train (BF16 forward and backward on the matrix
cores, Adam on FP32 master weights), class-weighted by the inverse square
root of the label counts.  The blob it returns is what bs_set_policy takes
for BS_POLICY_LEARNED.
"""
from __future__ import annotations

import time

import numpy as np

from . import (BS_POLICY_FIXED, bs_learn_pairs, bs_learn_sample_pairs, bs_mesh_free, bs_mesh_upload, bs_mlp_logits,
               bs_mlp_train, bs_set_policy)


def train(meshes, tau=0.01, pairs_per_mesh=100_000, epochs=30, batch=1024, lr=2e-3, seed=4, val_frac=0.1):
    """meshes: iterable of (xyz, omega, tets).  Returns (blob uint16 [5540],
    info dict: pairs, label counts, validation accuracy and majority share,
    final loss, seconds)."""
    import torch

    t0 = time.perf_counter()
    feats, labels = [], []
    for xyz, omega, tets in meshes:
        h = bs_mesh_upload(xyz, omega, tets)
        try:
            bs_set_policy(h, kind=BS_POLICY_FIXED)
            pairs = bs_learn_sample_pairs(h, pairs_per_mesh, seed)
            f, y, _ = bs_learn_pairs(h, pairs, tau)
            feats.append(f)
            labels.append(y)
        finally:
            bs_mesh_free(h)
    F = torch.cat(feats)
    Y = torch.cat(labels)
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
    info = {"pairs": int(Y.shape[0]), "label_counts": counts.astype(int).tolist(), "tau": tau, "epochs": epochs,
            "val_accuracy": float(np.mean(np.argmax(z, axis=1) == yv)),
            "val_majority": float(np.max(np.bincount(yv, minlength=4)) / max(1, len(yv))),
            "final_loss": float(losses[-1]) if len(losses) else None, "seconds": time.perf_counter() - t0}
    return blob, info
