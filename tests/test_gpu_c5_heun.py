"""Step 1 of the two-ring Lagrangian run at full size (80^3 Kuhn cells,
531,441 nodes, 3,072,000 tetrahedra) against the same Heun step taken by the
FP64 oracle alone (tests/golden/c5_heun_step1.json, written by
tests/golden/make_c5_heun_reference.py; the oracle's whole-mesh evaluation
takes hours, so it is stored).  Fixed distance rule, 16 x 16 lines, FP32
compensated on the GPU, dt = 0.005.

Tolerances: the velocity at the start, per sampled node, within 1e-6 of the
largest sampled speed (the library's stated bound); the positions after the
step within 1e-6 of the step's largest displacement at the sample (dt times
the speed: a velocity error e moves a node by at most dt e)."""
import json
import os

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
GOLDEN = os.path.join(HERE, "golden", "c5_heun_step1.json")


def _say(msg):
    print(msg, flush=True)


def test_c5_heun_step_one_matches_the_oracle():
    import torch

    assert torch.cuda.is_available()
    import paper_0712_1695_amd as bs

    with open(GOLDEN) as f:
        ref = json.load(f)
    nodes = np.asarray(ref["nodes"], dtype=np.int64)
    v1_ref, x1_ref = np.asarray(ref["v1"]), np.asarray(ref["x1"])
    dt = float(ref["dt"])
    m = W.make_config("C5")
    _say(f"C5 Heun step 1: {m.n_nodes} nodes, {m.n_tets} tets, {len(nodes)} sampled nodes, dt {dt}")
    h = bs.bs_mesh_upload(m.xyz, m.omega, m.tets)
    try:
        bs.bs_set_policy(h, kind=bs.BS_POLICY_FIXED)
        v1 = bs.bs_eval_velocity(h)[nodes]
        pos, secs = bs.bs_advect_heun(h, dt, 1)
    finally:
        bs.bs_mesh_free(h)
    x1 = pos[nodes]
    vscale = np.abs(v1_ref).max()
    ev = np.abs(v1 - v1_ref).max() / vscale
    ev_l2 = np.linalg.norm(v1 - v1_ref) / np.linalg.norm(v1_ref)
    step = np.abs(x1_ref - m.xyz[nodes]).max()
    ex = np.abs(x1 - x1_ref).max() / step
    _say(f"v1: max per-node error {ev:.3e} of the largest speed, rel-L2 {ev_l2:.3e}; "
         f"x1: max error {ex:.3e} of the largest displacement ({step:.3e}); step {secs[0]:.2f} s")
    assert ev <= 1e-6 and ev_l2 <= 1e-6
    assert ex <= 1e-6
