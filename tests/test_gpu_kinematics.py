"""The Lagrangian kinematics on the GPU against the oracle: the nodal
velocity gradient (bs_velocity_gradient) on seeded velocities, and Heun
steps that stretch the vorticity (bs_advect_heun with stretch) against the
same steps driven by the oracle in FP64."""
import numpy as np
import pytest

import oracle
import oracle.kinematics as K
import workloads as W

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def bs():
    import torch

    assert torch.cuda.is_available()
    import paper_0712_1695_amd as bs

    return bs


@pytest.mark.parametrize("name,scale", [("C1", (6, 6, 6)), ("C5", (9, 8, 10))])
def test_velocity_gradient_matches_oracle(bs, name, scale):
    m = W.make_config(name, scale=scale)
    _say(f"velocity gradient: {name} at {scale}, {m.n_nodes} nodes, {m.n_tets} tets")
    rng = np.random.default_rng(11)
    vel = rng.standard_normal((m.n_nodes, 3))
    h = bs.bs_mesh_upload(m.xyz, m.omega, m.tets)
    try:
        g = bs.bs_velocity_gradient(h, vel=vel)
        ref = K.nodal_velocity_gradient(m.xyz, m.tets, vel)
        err = np.max(np.abs(g - ref)) / np.max(np.abs(ref))
        _say(f"max |G - G_oracle| / max |G_oracle| = {err:.3e}")
        assert err <= 1e-9
        # a globally linear field comes back exactly (to rounding)
        A = rng.standard_normal((3, 3))
        gl = bs.bs_velocity_gradient(h, vel=m.xyz @ A.T + 0.3)
        assert np.max(np.abs(gl - A)) <= 1e-8 * np.max(np.abs(A))
    finally:
        bs.bs_mesh_free(h)


def test_stretching_rate_matches_oracle(bs):
    """bs_stretching_rate: G_i omega_i with the mesh's vorticity, against the
    oracle's gradient and stretching on seeded velocities; the last
    evaluation's velocities give the rate of that evaluation."""
    m = W.make_config("C5", scale=(9, 8, 10))
    vel = np.random.default_rng(12).standard_normal((m.n_nodes, 3))
    h = bs.bs_mesh_upload(m.xyz, m.omega, m.tets)
    try:
        r = bs.bs_stretching_rate(h, vel=vel)
        ref = K.stretching(K.nodal_velocity_gradient(m.xyz, m.tets, vel), m.omega)
        err = np.max(np.abs(r - ref)) / np.max(np.abs(ref))
        _say(f"stretching rate: max |s - s_oracle| / max |s_oracle| = {err:.3e}")
        assert err <= 1e-9
        v = bs.bs_eval_velocity(h)
        assert np.array_equal(bs.bs_stretching_rate(h), bs.bs_stretching_rate(h, vel=v))
    finally:
        bs.bs_mesh_free(h)


def test_gradient_of_the_last_evaluation(bs):
    m = W.make_config("C1", scale=(5, 5, 5))
    h = bs.bs_mesh_upload(m.xyz, m.omega, m.tets)
    try:
        with pytest.raises(bs.BsError) as ei:
            bs.bs_velocity_gradient(h)
        assert ei.value.status == bs.BS_E_STATE
        v = bs.bs_eval_velocity(h)
        assert np.array_equal(bs.bs_velocity_gradient(h), bs.bs_velocity_gradient(h, vel=v))
        bs.bs_mesh_update(h, xyz=m.xyz)  # new positions: no current velocities
        with pytest.raises(bs.BsError):
            bs.bs_velocity_gradient(h)
    finally:
        bs.bs_mesh_free(h)


def test_heun_with_stretching_matches_oracle(bs):
    """Two Heun steps of the two-ring workload (12^3 cells) moving the nodes
    and stretching their vorticity, against the oracle's steps (its own
    velocities, gradient and updates in FP64)."""
    m = W.make_config("C5", scale=(12, 12, 12))
    dt, steps = 0.02, 2
    _say(f"Lagrangian with stretching: {m.n_nodes} nodes, {steps} Heun steps")
    h = bs.bs_mesh_upload(m.xyz, m.omega, m.tets)
    try:
        pos, secs = bs.bs_advect_heun(h, dt, steps, stretch=True)
        x_gpu, w_gpu = bs.bs_mesh_read(h)
    finally:
        bs.bs_mesh_free(h)
    assert np.array_equal(pos, x_gpu)
    def run(perturb):
        rng = np.random.default_rng(21)

        def vel(xx, ww):
            v = oracle.evaluate(xx, ww, m.tets)
            if perturb:
                v = v + perturb * np.sqrt(np.mean(v * v)) * rng.standard_normal(v.shape)
            return v

        x, w = m.xyz.copy(), m.omega.copy()
        for _ in range(steps):
            x, w = K.lagrangian_step(x, w, m.tets, dt, vel)
        return x, w

    def errors(xa, wa, xb, wb):
        ex = np.linalg.norm((xa - m.xyz) - (xb - m.xyz)) / np.linalg.norm(xb - m.xyz)
        ew = np.linalg.norm((wa - m.omega) - (wb - m.omega)) / np.linalg.norm(wb - m.omega)
        return ex, ew

    x, w = run(0.0)
    # Tolerance from the conditioning of the step: every evaluation may err
    # by 1e-6 (rel-L2), and the nodal gradient turns velocity errors that vary
    # from node to node into stretching errors of order error / h.  The
    # oracle's own steps with i.i.d. velocity errors of rel-L2 1e-6 show how
    # much of that reaches the displacement and the vorticity change; the
    # library's steps may err by twice that.
    xp, wp = run(1e-6)
    ax, aw = errors(xp, wp, x, w)
    ex, ew = errors(x_gpu, w_gpu, x, w)
    _say(f"rel-L2 of displacement {ex:.3e}, of vorticity change {ew:.3e}; "
         f"from 1e-6 velocity noise: {ax:.3e}, {aw:.3e}")
    assert np.linalg.norm(w - m.omega) > 1e-3 * np.linalg.norm(m.omega)  # the vorticity did change
    assert ex <= max(1e-6, 2 * ax) and ew <= max(1e-6, 2 * aw)


def test_remeshed_run_and_parity_on_the_new_mesh(bs):
    """A run that stretches and re-tetrahedralises the points before every
    evaluation, then the velocity on a Delaunay mesh of its final nodes
    against the oracle on that mesh (the flat tets Qhull leaves on lattices
    are dropped, so the mesh has zero-volume cracks and takes the candidate
    ray kernel)."""
    from paper_0712_1695_amd.lagrangian import retetrahedralise, run

    m = W.make_config("C5", scale=(8, 8, 8))
    x, w, secs, _, last = run(m.xyz, m.omega, m.tets, 3, 0.02, stretch=True, remesh=True)
    _say(f"remeshed run: {len(secs)} steps, last mesh {last.shape[0]} tets")
    assert len(secs) == 3
    assert np.all(np.isfinite(x)) and np.all(np.isfinite(w))
    assert np.linalg.norm(w - m.omega) > 1e-3 * np.linalg.norm(m.omega)
    tets = retetrahedralise(x)
    h = bs.bs_mesh_upload(x, w, tets)
    try:
        v = bs.bs_eval_velocity(h)
    finally:
        bs.bs_mesh_free(h)
    ref = oracle.evaluate(x, w, tets)
    err = np.linalg.norm(v - ref) / np.linalg.norm(ref)
    _say(f"Delaunay mesh of the moved nodes ({tets.shape[0]} tets): rel-L2 vs oracle {err:.3e}")
    assert err <= 1e-6


def test_velocity_gradient_device_pointers(bs):
    """Device velocities and a device output give the host call's bits."""
    import torch

    m = W.make_config("C1", scale=(5, 6, 7))
    vel = np.random.default_rng(3).standard_normal((m.n_nodes, 3))
    h = bs.bs_mesh_upload(m.xyz, m.omega, m.tets)
    try:
        g_host = bs.bs_velocity_gradient(h, vel=vel)
        out = torch.empty((m.n_nodes, 3, 3), dtype=torch.float64, device="cuda")
        bs.bs_velocity_gradient(h, vel=torch.tensor(vel, device="cuda"), out=out)
        torch.cuda.synchronize()
        assert np.array_equal(out.cpu().numpy(), g_host)
    finally:
        bs.bs_mesh_free(h)
