"""bs_eval_velocity_noalloc (for callers that cannot allocate device memory)
through the C ABI: its velocities against bs_eval_velocity's on the same
mesh, on two calls in a row (the second with a smaller mesh, so that the
static scratch holds the first call's contents), for the fixed and learned
policies, the vector-ALU far field and the treecode far field; a mesh too
large for the scratch is refused before anything runs."""
import ctypes
import json
import os

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

TOL = 1e-6
HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def bs():
    import torch

    assert torch.cuda.is_available()
    torch.cuda.set_device(0)
    import paper_0712_1695_amd as bs

    return bs


def _both(bs, m, pol, valu_far=False):
    import torch

    h = bs.bs_mesh_upload(m.xyz, m.omega, m.tets)
    try:
        bs.bs_set_policy(h, **pol)
        ref = bs.bs_eval_velocity(h, valu_far=valu_far)
        out = torch.full((m.n_nodes, 3), float("nan"), dtype=torch.float64, device="cuda")
        L = bs.load_library()
        flags = bs.BS_PTR_DEVICE | (bs.BS_EVAL_VALU_FAR if valu_far else 0)
        stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
        rc = L.bs_eval_velocity_noalloc(h.handle, ctypes.c_void_p(out.data_ptr()), flags, stream)
        assert rc == bs.BS_OK, L.bs_last_error().decode()
        torch.cuda.synchronize()
        v = out.cpu().numpy()
    finally:
        bs.bs_mesh_free(h)
    return v, ref


def _check(v, ref, label):
    e = float(np.linalg.norm(v - ref) / np.linalg.norm(ref))
    print(f"{label}: rel-L2 vs bs_eval_velocity {e:.3e}, bitwise equal {np.array_equal(v, ref)}", flush=True)
    assert np.all(np.isfinite(v))
    assert e <= TOL


def test_noalloc_matches_eval_velocity_two_calls(bs):
    blob = json.load(open(os.path.join(HERE, "golden", "selector_blob.json")))
    bits = np.array(blob["blob_bf16_bits"], dtype=np.uint16)
    cases = [("fixed", dict(kind=bs.BS_POLICY_FIXED), False),
             ("fixed, vector-ALU far field", dict(kind=bs.BS_POLICY_FIXED), True),
             ("learned", dict(kind=bs.BS_POLICY_LEARNED, mlp_bf16=bits, conf_min=float(blob["conf_min"])), False),
             ("pure ray tracing 8x12", dict(kind=bs.BS_POLICY_PURE_RT, n_phi=8, n_theta=12), False),
             ("fixed, treecode far field", dict(kind=bs.BS_POLICY_FIXED, near_cut=1.0, d_g11=1.5, d_g4=2.0,
                                                far_field="treecode", tree_theta=0.5, tree_order=4), False)]
    for label, pol, valu in cases:
        for cells in ((12, 11, 10), (5, 6, 4)):  # second call smaller: the scratch keeps the first's contents
            m = W.make_config("C1", scale=cells)
            v, ref = _both(bs, m, pol, valu)
            _check(v, ref, f"{label}, C1 at {cells} ({m.n_nodes} nodes)")


def test_noalloc_where_the_boundary_is_not_convex(bs):
    """Meshes whose boundary is not convex (the ball clipped from Kuhn
    cells; the cube with displaced boundary nodes): the walk leaves nodes to
    the candidate kernel through the node list in the static scratch, and
    the learned policy's selection lists live there too."""
    blob = json.load(open(os.path.join(HERE, "golden", "selector_blob.json")))
    bits = np.array(blob["blob_bf16_bits"], dtype=np.uint16)
    learned = dict(kind=bs.BS_POLICY_LEARNED, mlp_bf16=bits, conf_min=float(blob["conf_min"]))
    ball = W.ball_mesh(cells=12)
    ball.omega = W.field_gaussian_swirl(ball.xyz)
    cube = W.make_config("C1", scale=(8, 8, 8))
    rng = np.random.default_rng(31)
    cube.xyz = cube.xyz.copy()
    cube.xyz[cube.boundary] += rng.uniform(-0.05, 0.05, size=(int(cube.boundary.sum()), 3)) * cube.h
    for label, pol in (("fixed", dict(kind=bs.BS_POLICY_FIXED)), ("learned", learned)):
        for name, m in (("ball", ball), ("displaced cube", cube)):  # second call smaller
            v, ref = _both(bs, m, pol)
            _check(v, ref, f"{label}, {name} ({m.xyz.shape[0]} nodes)")


def test_noalloc_refuses_meshes_beyond_the_scratch(bs):
    """A host output, and the learned policy on the ring workload (97,175
    nodes: 24 bytes x 8 splits + 48 per node slot and 532 per node, 75 MB),
    are refused before any kernel runs."""
    import torch

    L = bs.load_library()
    blob = json.load(open(os.path.join(HERE, "golden", "selector_blob.json")))
    bits = np.array(blob["blob_bf16_bits"], dtype=np.uint16)
    big = W.make_config("C2")
    hb = bs.bs_mesh_upload(big.xyz, big.omega, big.tets)
    try:
        outb = torch.empty((big.n_nodes, 3), dtype=torch.float64, device="cuda")
        assert L.bs_eval_velocity_noalloc(hb.handle, ctypes.c_void_p(outb.data_ptr()), 0, None) == bs.BS_E_ARG
        bs.bs_set_policy(hb, kind=bs.BS_POLICY_LEARNED, mlp_bf16=bits, conf_min=float(blob["conf_min"]))
        rc = L.bs_eval_velocity_noalloc(hb.handle, ctypes.c_void_p(outb.data_ptr()), bs.BS_PTR_DEVICE, None)
        msg = L.bs_last_error().decode()
        print(f"learned on the ring (97,175 nodes): status {rc}: {msg}", flush=True)
        assert rc == bs.BS_E_ARG and "scratch" in msg
    finally:
        bs.bs_mesh_free(hb)
