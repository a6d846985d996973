"""Lagrangian run of the two-ring workload through bs_advect_heun.

The paper's application (Sections 1 and 3): control points carrying
vorticity move with the flow and their velocities are re-evaluated each
step.  By default connectivity and nodal vorticity are kept.  With
--stretch the nodal vorticity is also advanced by vortex stretching,
(w . grad) v with the nodal velocity gradient of the library; with
--remesh the points are re-tetrahedralised before every evaluation (a
Delaunay tetrahedralisation by Qhull through scipy, on the host, where the
paper uses the external TetGen mesher), so a run can go on past the point
where the original connectivity would fold.  Every evaluation runs in the
library: FP64 Heun updates on the host, per-element precompute, two device
evaluations (and with --stretch two gradient passes) per step.

    python -m paper_0712_1695_amd.lagrangian --steps 10 --dt 0.005 --stretch --remesh
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

from . import (BS_POLICY_FIXED, BS_PREC_FP32_COMP, bs_advect_heun, bs_eval_velocity, bs_mesh_free, bs_mesh_read,
               bs_mesh_upload, bs_set_policy, bs_stretching_rate)


def retetrahedralise(xyz, min_quality=1e-6):
    """Delaunay tetrahedra of the points (Qhull), positively oriented,
    without the flat ones Qhull returns for co-spherical points (volume
    below min_quality times the longest edge cubed; such tets hold no
    volume, so the union still fills the convex hull).  Returns int32 [T,4]."""
    from scipy.spatial import Delaunay

    xyz = np.asarray(xyz, dtype=np.float64)
    tets = Delaunay(xyz).simplices.astype(np.int32)
    X = xyz[tets]
    det = np.linalg.det(X[:, 1:, :] - X[:, :1, :])
    edge = np.max(np.linalg.norm(X[:, :, None, :] - X[:, None, :, :], axis=-1).reshape(len(tets), -1), axis=1)
    keep = np.abs(det) > min_quality * edge ** 3
    tets = tets[keep]
    flip = det[keep] < 0
    tets[flip, 2], tets[flip, 3] = tets[flip, 3].copy(), tets[flip, 2].copy()
    return tets


def _stage(x, w, policy, stretch):
    """One evaluation on a fresh tetrahedralisation of the points x:
    (velocity, stretching rate or None, tets)."""
    tets = retetrahedralise(x)
    h = bs_mesh_upload(x, w, tets)
    try:
        bs_set_policy(h, **policy)
        v = bs_eval_velocity(h)
        s = bs_stretching_rate(h) if stretch else None
        return v, s, tets
    finally:
        bs_mesh_free(h)


def run(xyz, omega, tets, steps, dt, policy=None, stretch=False, remesh=False):
    """Returns (final positions, final vorticity, per-step seconds,
    first-step velocity, tets of the last tetrahedralisation).  Without
    remesh the connectivity is kept (bs_advect_heun); with remesh every
    evaluation runs on a Delaunay tetrahedralisation of the current points
    (the paper's setting: the points are tetrahedralised at each step, here
    at each Heun stage too, so no element can fold)."""
    policy = policy or dict(kind=BS_POLICY_FIXED, precision=BS_PREC_FP32_COMP)
    if not remesh:
        h = bs_mesh_upload(xyz, omega, tets)
        try:
            bs_set_policy(h, **policy)
            v1 = bs_eval_velocity(h)
            _, secs = bs_advect_heun(h, dt, steps, stretch=stretch)
            x, w = bs_mesh_read(h)
            return x, w, secs, v1, tets
        finally:
            bs_mesh_free(h)
    x = np.asarray(xyz, dtype=np.float64).copy()
    w = np.asarray(omega, dtype=np.float64).copy()
    secs, v_first = [], None
    for _ in range(steps):
        t0 = time.perf_counter()
        v1, s1, _ = _stage(x, w, policy, stretch)
        if v_first is None:
            v_first = v1
        xs = x + dt * v1
        ws = w + dt * s1 if stretch else w
        v2, s2, t_last = _stage(xs, ws, policy, stretch)
        x = x + 0.5 * dt * (v1 + v2)
        if stretch:
            w = w + 0.5 * dt * (s1 + s2)
        secs.append(time.perf_counter() - t0)
    return x, w, np.array(secs), v_first, t_last


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--dt", type=float, default=0.005)
    ap.add_argument("--cells", type=int, default=80)
    ap.add_argument("--learned", action="store_true", help="learned policy (selector trained on the GPU first)")
    ap.add_argument("--stretch", action="store_true", help="advance the nodal vorticity by vortex stretching")
    ap.add_argument("--remesh", action="store_true", help="re-tetrahedralise the points before every evaluation")
    args = ap.parse_args()
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    if root not in sys.path:
        sys.path.insert(0, root)
    import workloads as W

    m = W.make_config("C5", scale=None if args.cells == 80 else (args.cells,) * 3)
    policy = dict(kind=BS_POLICY_FIXED, precision=BS_PREC_FP32_COMP)
    sel = None
    if args.learned:
        from . import BS_POLICY_LEARNED, selector

        blob, sel = selector.train_selector(W.make_config, held_out=())
        policy = dict(kind=BS_POLICY_LEARNED, precision=BS_PREC_FP32_COMP, mlp_bf16=blob, conf_min=0.9)
    pos, om, secs, _, last = run(m.xyz, m.omega, m.tets, args.steps, args.dt, policy, stretch=args.stretch,
                                 remesh=args.remesh)
    disp = np.linalg.norm(pos - m.xyz, axis=1)
    print(json.dumps({"workload": m.name, "nodes": m.n_nodes, "tets": m.n_tets, "steps": args.steps, "dt": args.dt,
                      "policy": "learned" if args.learned else "fixed", "stretch": args.stretch,
                      "pairs_per_eval": m.n_nodes * m.n_tets, "evals": 2 * args.steps,
                      "step_seconds": [float(s) for s in secs], "max_displacement": float(disp.max()),
                      "vorticity_change": float(np.linalg.norm(om - m.omega) / np.linalg.norm(m.omega)),
                      "remesh": args.remesh, "tets_last": int(last.shape[0]),
                      "selector": sel}), flush=True)


if __name__ == "__main__":
    main()
