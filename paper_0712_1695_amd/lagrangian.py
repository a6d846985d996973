"""Lagrangian run of the two-ring workload through bs_advect_heun.

The paper's application (Sections 1 and 3): control points carrying
vorticity move with the flow and their velocities are re-evaluated each
step.  Connectivity and nodal vorticity are kept (the paper
re-tetrahedralises with an external mesher).  Every step runs in the
library: FP64 Heun updates on the host, per-element precompute, and two
device evaluations.

    python -m paper_0712_1695_amd.lagrangian --steps 10 --dt 0.005
"""
from __future__ import annotations

import argparse
import json
import os
import sys

import numpy as np

from . import (BS_POLICY_FIXED, BS_PREC_FP32_COMP, bs_advect_heun, bs_eval_velocity, bs_mesh_free, bs_mesh_upload,
               bs_set_policy)


def run(xyz, omega, tets, steps, dt, policy=None):
    """Returns (final positions, per-step seconds, first-step velocity)."""
    h = bs_mesh_upload(xyz, omega, tets)
    try:
        bs_set_policy(h, **(policy or dict(kind=BS_POLICY_FIXED, precision=BS_PREC_FP32_COMP)))
        v1 = bs_eval_velocity(h)
        pos, secs = bs_advect_heun(h, dt, steps)
        return pos, secs, v1
    finally:
        bs_mesh_free(h)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--dt", type=float, default=0.005)
    ap.add_argument("--cells", type=int, default=80)
    ap.add_argument("--learned", action="store_true", help="learned policy (selector trained on the GPU first)")
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

        tm = [W.make_config("C1"), W.make_config("C2", scale=(32, 32, 11))]
        blob, sel = selector.train([(t.xyz, t.omega, t.tets) for t in tm])
        policy = dict(kind=BS_POLICY_LEARNED, precision=BS_PREC_FP32_COMP, mlp_bf16=blob, conf_min=0.9)
    pos, secs, _ = run(m.xyz, m.omega, m.tets, args.steps, args.dt, policy)
    disp = np.linalg.norm(pos - m.xyz, axis=1)
    print(json.dumps({"workload": m.name, "nodes": m.n_nodes, "tets": m.n_tets, "steps": args.steps, "dt": args.dt,
                      "policy": "learned" if args.learned else "fixed",
                      "pairs_per_eval": m.n_nodes * m.n_tets, "evals": 2 * args.steps,
                      "step_seconds": [float(s) for s in secs], "max_displacement": float(disp.max()),
                      "selector": sel}), flush=True)


if __name__ == "__main__":
    main()
