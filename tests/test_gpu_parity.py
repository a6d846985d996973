"""GPU parity: the HIP library (through the C ABI) against the FP64 oracle
on the same seeded inputs.

Tolerance: relative L2 error <= 1e-6 over all nodes and components for the
FP32 path (the stated target), per policy, and at every node an error at
most 5e-6 of the larger of the node's own velocity and the root-mean-square
node velocity (so that one bad node cannot hide in the aggregate; the floor
keeps nodes whose velocity nearly cancels from dominating).  Rule decisions
(binary32 on both sides) must match exactly, pair counts included."""
import json
import os

import numpy as np
import pytest

import oracle
from oracle import references as R
import paper_0712_1695_amd as bs
import workloads as W

pytestmark = pytest.mark.gpu

TOL = 1e-6
NODE_TOL = 5e-6


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a device"
    torch.cuda.set_device(0)


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def node_errors(a, b):
    """Per-node error relative to max(|b_i|, rms node magnitude of b)."""
    scale = np.sqrt(np.mean(np.sum(b * b, axis=1)))
    return np.linalg.norm(a - b, axis=1) / np.maximum(np.linalg.norm(b, axis=1), max(scale, 1e-300))


def check(a, b, label="", tol=TOL, node_tol=NODE_TOL):
    """Assert rel-L2 <= tol and the per-node bound; print both."""
    e = rel_l2(a, b)
    per = node_errors(a, b)
    _say(f"  {label} rel-L2 {e:.3e}, worst node {per.max():.3e} (of {len(per)})")
    assert e <= tol, (label, e)
    assert per.max() <= node_tol, (label, per.max(), int(per.argmax()))
    return e


def gpu_eval(mesh_or_arrays, **pol):
    if isinstance(mesh_or_arrays, W.Mesh):
        xyz, om, tets = mesh_or_arrays.xyz, mesh_or_arrays.omega, mesh_or_arrays.tets
    else:
        xyz, om, tets = mesh_or_arrays
    h = bs.bs_mesh_upload(xyz, om, tets)
    bs.bs_set_policy(h, **pol)
    v, st = bs.bs_eval_velocity(h, stats=True)
    bs.bs_mesh_free(h)
    return v, st


def _say(msg):
    print(msg, flush=True)


@pytest.mark.parametrize("rule,pts", [(0, 1), (1, 4), (2, 11)])
def test_gauss_only_c1(rule, pts):
    m = W.make_config("C1")
    _say(f"gauss-only G{pts} on C1")
    v, st = gpu_eval(m, kind=bs.BS_POLICY_GAUSS_ONLY, gauss_rule=rule)
    ref = oracle.evaluate(m.xyz, m.omega, m.tets, oracle.make_policy("gauss_only", gauss_rule=rule))
    check(v, ref, f"G{pts}")
    assert st["pairs_by_rule"][rule] == m.n_nodes * m.n_tets


@pytest.mark.parametrize("prec", [bs.BS_PREC_FP32_NAIVE, bs.BS_PREC_FP32_COMP, bs.BS_PREC_FP64])
def test_fixed_policy_c1(prec):
    m = W.make_config("C1")
    _say(f"fixed policy on C1, precision {prec}")
    v, st = gpu_eval(m, kind=bs.BS_POLICY_FIXED, precision=prec)
    ref, cnt = oracle.evaluate(m.xyz, m.omega, m.tets, oracle.make_policy("fixed"), return_counters=True)
    assert st["hbar"] == cnt["hbar"]
    assert st["pairs_by_rule"] == cnt["pairs_by_rule"]
    assert st["rt_hit_lines"] > 0
    assert st["nonfinite_out"] == 0
    check(v, ref, f"precision {prec}", node_tol=NODE_TOL if prec else 5e-5)


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("cells", [(10, 10, 10), (13, 14, 15)])
def test_far_field_matrix_and_vector_kernels(prec, cells):
    """The far field on the matrix cores (only the G1 pairs, block-centred
    FP32 contractions) and on the vector ALUs (every pair by G1, then the
    non-G1 pairs' terms removed) both match the oracle.  13 x 14 x 15 cells:
    3,360 nodes (a ragged last block of 32) and 16,380 tets (8 tet splits,
    the last one ragged)."""
    m = W.make_config("C1", scale=cells)
    _say(f"far-field kernels on C1 {cells}, precision {prec}")
    ref = oracle.evaluate(m.xyz, m.omega, m.tets, oracle.make_policy("fixed"))
    h = bs.bs_mesh_upload(m.xyz, m.omega, m.tets)
    bs.bs_set_policy(h, kind=bs.BS_POLICY_FIXED, precision=prec)
    v_m = bs.bs_eval_velocity(h)
    v_v = bs.bs_eval_velocity(h, valu_far=True)
    bs.bs_mesh_free(h)
    check(v_m, ref, "matrix cores", tol=TOL if prec else 1e-5, node_tol=NODE_TOL if prec else 5e-5)
    check(v_v, ref, "vector ALUs", tol=TOL if prec else 1e-5, node_tol=NODE_TOL if prec else 5e-5)


@pytest.mark.parametrize("nm", [(16, 16), (8, 12), (5, 7)])
def test_pure_ray_tracing_c1(nm):
    """Odd orders put a Gauss node at t = 0: lines with phi = pi/2 or
    theta = pi/2 are tangent to the box faces, and from an (unjittered)
    boundary node such a line runs along boundary faces, where the chord has
    no unique value (the line integral jumps between the two sides).  For
    odd orders only interior nodes are compared here; the general-position
    case is covered by the next test."""
    m = W.make_config("C1")
    _say(f"pure ray tracing on C1, N x M = {nm}")
    v, st = gpu_eval(m, kind=bs.BS_POLICY_PURE_RT, n_phi=nm[0], n_theta=nm[1])
    ref, cnt = oracle.evaluate(m.xyz, m.omega, m.tets, oracle.make_policy("pure_rt", n_phi=nm[0], n_theta=nm[1]),
                               return_counters=True)
    if nm[0] % 2 or nm[1] % 2:
        keep = ~m.boundary
        assert np.all(np.isfinite(v))
        check(v[keep], ref[keep], "interior nodes")
    else:
        check(v, ref, "all nodes")
        # every (line, tet) hit of the oracle is one ray hit on the GPU (exact
        # decisions away from edges and vertices; allow a few near-edge flips)
        assert abs(st["rt_hit_lines"] - cnt["rt_hit_lines"]) <= 1e-5 * cnt["rt_hit_lines"] + 8


@pytest.mark.parametrize("nm", [(5, 7), (3, 3), (16, 16)])
def test_pure_ray_tracing_general_position(nm):
    """Every node jittered (boundary included): no line lies in a face plane,
    so the result is unique for any order and all nodes are compared."""
    xyz, tets, h, b = W.kuhn_grid((-1, -1, -1), (1, 1, 1), (7, 6, 5))
    xyz = xyz + np.random.default_rng(9).uniform(-0.1, 0.1, size=xyz.shape) * h[None, :]
    tets = W.orient_positive(xyz, tets)
    om = W.field_gaussian_swirl(xyz)
    _say(f"pure ray tracing, general position, N x M = {nm}")
    v, _ = gpu_eval((xyz, om, tets), kind=bs.BS_POLICY_PURE_RT, n_phi=nm[0], n_theta=nm[1])
    ref = oracle.evaluate(xyz, om, tets, oracle.make_policy("pure_rt", n_phi=nm[0], n_theta=nm[1]))
    check(v, ref, f"{nm}")


def test_ring_reduced_full_oracle():
    m = W.make_config("C2", scale=(24, 24, 8))
    _say(f"ring at 24x24x8 cells ({m.n_nodes} nodes), fixed policy")
    v, st = gpu_eval(m)
    ref, cnt = oracle.evaluate(m.xyz, m.omega, m.tets, oracle.make_policy("fixed"), return_counters=True)
    assert st["pairs_by_rule"] == cnt["pairs_by_rule"]
    check(v, ref, "ring 24x24x8")


def _sample_nodes(m, k, seed):
    rng = np.random.default_rng(seed)
    corners = [0, m.n_nodes - 1]
    inner = rng.choice(m.n_nodes, size=k - 2, replace=False)
    return np.unique(np.concatenate([corners, inner]))


@pytest.mark.parametrize("name", ["C2", "C3", "C5"])
def test_full_size_sampled(name):
    """Full workload on the GPU in the configuration the benchmark times;
    the oracle evaluates a seeded sample of nodes one by one."""
    m = W.make_config(name)
    _say(f"{name} full size ({m.n_nodes} nodes, {m.n_tets} tets), fixed policy")
    v, st = gpu_eval(m)
    tg = _sample_nodes(m, 256, seed=11)
    ref = oracle.evaluate(m.xyz, m.omega, m.tets, oracle.make_policy("fixed"), targets=tg)
    _say(f"{name}: rules {st['pairs_by_rule']}; t_eval {st['t_eval_s']*1e3:.2f} ms")
    check(v[tg], ref, f"{name} {len(tg)} sampled nodes")
    assert sum(st["pairs_by_rule"]) == m.n_nodes * m.n_tets


def test_precision_modes_c3_sampled():
    """Precision sweep on the 48^3 Fourier-curl workload, for both far-field
    kernels; errors reported per result (whole-sample rel-L2, worst node).
    Compensated and FP64 accumulation stay within 1e-6, and within 3e-7 on
    this sample (measured 1.2e-7 to 1.5e-7: no kernel sums more than 32
    tets' terms in FP32 before a compensated or FP64 fold; summing whole
    bin rows held every mode near 5e-7).  Naive accumulation
    is one FP32 sum per node and tet split on the vector ALUs (past 1e-6
    there); the matrix-core kernel adds FP32 sums of its eight splits in
    FP64 even then."""
    m = W.make_config("C3")
    tg = _sample_nodes(m, 256, seed=3)
    ref = oracle.evaluate(m.xyz, m.omega, m.tets, oracle.make_policy("fixed"), targets=tg)
    h = bs.bs_mesh_upload(m.xyz, m.omega, m.tets)
    for valu in (False, True):
        errs = {}
        for prec in (bs.BS_PREC_FP32_NAIVE, bs.BS_PREC_FP32_COMP, bs.BS_PREC_FP64):
            bs.bs_set_policy(h, kind=bs.BS_POLICY_FIXED, precision=prec)
            v, st = bs.bs_eval_velocity(h, stats=True, valu_far=valu)
            err = rel_l2(v[tg], ref)
            per = node_errors(v[tg], ref)
            _say(f"C3 precision {prec}, {'vector ALUs' if valu else 'matrix cores'}: rel-L2 {err:.3e}, "
                 f"worst node {per.max():.3e}, t_eval {st['t_eval_s']*1e3:.1f} ms")
            errs[prec] = err
            if prec != bs.BS_PREC_FP32_NAIVE:
                assert per.max() <= NODE_TOL, (prec, valu, per.max())
        assert errs[bs.BS_PREC_FP32_COMP] <= TOL and errs[bs.BS_PREC_FP64] <= TOL
        assert errs[bs.BS_PREC_FP32_COMP] <= 3e-7 and errs[bs.BS_PREC_FP64] <= 3e-7
        assert errs[bs.BS_PREC_FP32_NAIVE] <= 1e-4
        if valu:
            assert errs[bs.BS_PREC_FP32_NAIVE] > errs[bs.BS_PREC_FP32_COMP]
    bs.bs_mesh_free(h)


# ------------------------------------------------------------------ edges

def test_single_tet_and_tiny_meshes():
    t = W.single_tet(5)
    for kind in (bs.BS_POLICY_FIXED, bs.BS_POLICY_PURE_RT):
        v, _ = gpu_eval(t, kind=kind)
        ref = oracle.evaluate(t.xyz, t.omega, t.tets,
                              oracle.make_policy("fixed" if kind == bs.BS_POLICY_FIXED else "pure_rt"))
        check(v, ref, f"single tet, policy {kind}")
    m = W.make_config("C1", scale=(1, 1, 1))
    v, _ = gpu_eval(m)
    check(v, oracle.evaluate(m.xyz, m.omega, m.tets), "one cell")


def test_no_tets_gives_zero_velocity():
    xyz = np.random.default_rng(0).standard_normal((37, 3))
    v, st = gpu_eval((xyz, np.ones((37, 3)), np.zeros((0, 4), dtype=np.int32)))
    assert np.all(v == 0.0) and st["pairs"] == 0


def test_ragged_counts_and_unreferenced_nodes():
    """Node count not a multiple of any block size; extra nodes used by no
    tetrahedron (their velocity is still evaluated), some of them inside
    tetrahedra (off-node targets: rays start inside the element)."""
    m = W.make_config("C1", scale=(3, 5, 4))
    rng = np.random.default_rng(2)
    extra = rng.uniform(-1.5, 1.5, size=(7, 3))
    xyz = np.vstack([m.xyz, extra])
    om = np.vstack([m.omega, rng.standard_normal((7, 3))])
    v, st = gpu_eval((xyz, om, m.tets))
    ref, cnt = oracle.evaluate(xyz, om, m.tets, return_counters=True)
    assert st["pairs_by_rule"] == cnt["pairs_by_rule"]
    check(v, ref, "ragged")


def test_reoriented_tets():
    m = W.make_config("C1", scale=(4, 4, 4))
    tets = m.tets.copy()
    flip = np.arange(0, m.n_tets, 3)
    tets[flip, 1], tets[flip, 2] = m.tets[flip, 2], m.tets[flip, 1]
    v, st = gpu_eval((m.xyz, m.omega, tets))
    assert st["reoriented"] == flip.size
    check(v, oracle.evaluate(m.xyz, m.omega, tets), "reoriented")


@pytest.mark.parametrize("name,scale,valu", [("C1", None, False), ("C1", None, True),
                                             ("C2", (24, 24, 8), False)])
def test_incident_pairs_beyond_the_cuts(name, scale, valu):
    """Cuts below the largest vertex-centroid distance (ray tracing below
    0.5, G11 below 0.65, G4 below 0.8 mean edge lengths; the largest
    vertex-centroid distance is 0.86 of it on C1): a tet having the node as
    a vertex can lie beyond every cut, so the far-field and band kernels take
    their incidence tests (the rule ray-traces every incident pair), on the
    matrix-core and on the vector-ALU far field."""
    m = W.make_config(name) if scale is None else W.make_config(name, scale=scale)
    cuts = dict(near_cut=0.5, d_g11=0.65, d_g4=0.8)
    hb = oracle.mean_edge(m.xyz, m.tets)
    X = m.xyz[m.tets]
    vc = np.linalg.norm(X - X.mean(axis=1)[:, None, :], axis=2)
    assert (vc > cuts["d_g4"] * hb).sum() > 0  # incident pairs beyond the G4 cut exist
    _say(f"{name} {m.n_nodes} nodes, cuts {cuts}, {'vector ALUs' if valu else 'matrix cores'}; "
         f"{(vc > cuts['d_g4'] * hb).sum()} vertex-tet pairs beyond the G4 cut")
    h = bs.bs_mesh_upload(m.xyz, m.omega, m.tets)
    try:
        bs.bs_set_policy(h, kind=bs.BS_POLICY_FIXED, **cuts)
        v, st = bs.bs_eval_velocity(h, stats=True, valu_far=valu)
    finally:
        bs.bs_mesh_free(h)
    ref, cnt = oracle.evaluate(m.xyz, m.omega, m.tets, oracle.make_policy("fixed", **cuts),
                               return_counters=True)
    _say(f"  rules {st['pairs_by_rule']} (oracle {cnt['pairs_by_rule']})")
    assert st["pairs_by_rule"] == cnt["pairs_by_rule"]
    check(v, ref, "incident beyond cuts")


def test_device_pointers_update_stream_and_determinism():
    import torch

    m = W.make_config("C1", scale=(6, 6, 6))
    dev = torch.device("cuda", 0)
    xyz_t = torch.tensor(m.xyz, device=dev)
    om_t = torch.tensor(m.omega, device=dev)
    tets_t = torch.tensor(m.tets, device=dev)
    h_host = bs.bs_mesh_upload(m.xyz, m.omega, m.tets)
    h_dev = bs.bs_mesh_upload(xyz_t, om_t, tets_t)
    a = bs.bs_eval_velocity(h_host)
    out = torch.empty((m.n_nodes, 3), dtype=torch.float64, device=dev)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        bs.bs_eval_velocity(h_dev, out=out)
    s.synchronize()
    assert np.array_equal(a, out.cpu().numpy())
    assert np.array_equal(a, bs.bs_eval_velocity(h_host))  # deterministic
    # update to other coordinates == fresh upload of those coordinates
    m2 = W.make_config("C1", scale=(6, 6, 6), seed=77)
    bs.bs_mesh_update(h_host, xyz=m2.xyz, omega=m2.omega)
    h2 = bs.bs_mesh_upload(m2.xyz, m2.omega, m2.tets)
    assert np.array_equal(bs.bs_eval_velocity(h_host), bs.bs_eval_velocity(h2))
    for h in (h_host, h_dev, h2):
        bs.bs_mesh_free(h)


def test_lagrangian_heun_matches_oracle_heun():
    """Two Heun steps of the two-ring workload (reduced to 12^3 cells):
    library (bs_advect_heun) against the same steps driven by the oracle in
    FP64.  Drift is measured on the displacement."""
    m = W.make_config("C5", scale=(12, 12, 12))
    dt, steps = 0.02, 2
    _say(f"Lagrangian: {m.n_nodes} nodes, {steps} Heun steps")
    h = bs.bs_mesh_upload(m.xyz, m.omega, m.tets)
    pos, secs, st = bs.bs_advect_heun(h, dt, steps, stats=True)
    bs.bs_mesh_free(h)
    x = m.xyz.copy()
    for _ in range(steps):
        v1 = oracle.evaluate(x, m.omega, m.tets)
        xs = x + dt * v1
        v2 = oracle.evaluate(xs, m.omega, m.tets)
        x = x + 0.5 * dt * (v1 + v2)
    disp_ref = x - m.xyz
    err = float(np.linalg.norm((pos - m.xyz) - disp_ref) / np.linalg.norm(disp_ref))
    _say(f"Lagrangian drift: rel-L2 of displacement {err:.3e}; step seconds {secs}")
    assert len(secs) == steps and np.all(secs > 0)
    # the displacement is dt/2 (v1 + v2) summed over the steps: its relative
    # error is bounded by the evaluations' (1e-6) up to the tiny change of
    # v2 with the positions
    assert err <= TOL


def test_lagrangian_reports_inversion():
    """A step large enough to fold the mesh stops with the offending tet and
    leaves the mesh at the start of that step."""
    m = W.make_config("C5", scale=(6, 6, 6))
    h = bs.bs_mesh_upload(m.xyz, m.omega, m.tets)
    v0 = bs.bs_eval_velocity(h)
    with pytest.raises(bs.BsError) as ei:
        bs.bs_advect_heun(h, 50.0, 1)
    assert ei.value.status == bs.BS_E_DEGENERATE
    assert np.array_equal(bs.bs_eval_velocity(h), v0)
    bs.bs_mesh_free(h)


def test_walk_and_candidate_kernels_agree():
    """Ray tracing by walking face neighbours and by testing candidate rays
    per pair compute the same chords; both match the oracle.  On the convex
    cube every node walks; on the ball clipped from Kuhn cells (a staircase
    boundary) the nodes whose rays leave the mesh before their last
    ray-traced tet take the candidate kernel."""
    m = W.make_config("C1")
    ref = oracle.evaluate(m.xyz, m.omega, m.tets, oracle.make_policy("pure_rt"))
    v, st = gpu_eval(m, kind=bs.BS_POLICY_PURE_RT)
    check(v, ref, "walk")
    assert st["rt_walk_nodes"] == m.n_nodes and st["rt_candidate_nodes"] == 0
    b = W.ball_mesh(cells=12)
    b.omega = W.field_gaussian_swirl(b.xyz)
    vb, stb = gpu_eval(b)
    _say(f"  ball: {stb['rt_walk_nodes']} nodes walked, {stb['rt_candidate_nodes']} by candidate rays")
    check(vb, oracle.evaluate(b.xyz, b.omega, b.tets), "walk and candidate kernel on the ball")
    assert stb["rt_walk_nodes"] > 0 and stb["rt_candidate_nodes"] > 0
    assert stb["rt_walk_nodes"] + stb["rt_candidate_nodes"] == b.xyz.shape[0]


def test_walk_where_the_boundary_is_not_convex():
    """The cube with its boundary nodes displaced by up to 0.05 h (as a
    Lagrangian step leaves it: no longer convex).  Fixed rule: interior
    nodes walk, nodes with a ray that exits before its last ray-traced tet
    take candidate rays; pure ray tracing (rays to the boundary): every node
    takes candidate rays.  Both against the oracle."""
    m = W.make_config("C1")
    rng = np.random.default_rng(31)
    xyz = m.xyz.copy()
    nb = int(m.boundary.sum())
    xyz[m.boundary] += rng.uniform(-0.05, 0.05, size=(nb, 3)) * m.h
    arrays = (xyz, m.omega, m.tets)
    v, st = gpu_eval(arrays)
    _say(f"  displaced boundary: {st['rt_walk_nodes']} nodes walked, {st['rt_candidate_nodes']} by candidate rays")
    check(v, oracle.evaluate(xyz, m.omega, m.tets), "fixed rule, displaced boundary")
    assert st["rt_walk_nodes"] > 0 and st["rt_candidate_nodes"] >= nb
    vp, stp = gpu_eval(arrays, kind=bs.BS_POLICY_PURE_RT, n_phi=8, n_theta=8)
    check(vp, oracle.evaluate(xyz, m.omega, m.tets, oracle.make_policy("pure_rt", n_phi=8, n_theta=8)),
          "pure ray tracing, displaced boundary")
    assert stp["rt_walk_nodes"] == 0 and stp["rt_candidate_nodes"] == m.n_nodes


def test_concurrent_and_serial_streams_agree():
    """The band and ray-tracing kernels on the mesh's own streams give the
    same bits as every kernel on one stream."""
    m = W.make_config("C1", scale=(12, 12, 12))
    h = bs.bs_mesh_upload(m.xyz, m.omega, m.tets)
    for kind in (bs.BS_POLICY_FIXED, bs.BS_POLICY_PURE_RT):
        bs.bs_set_policy(h, kind=kind)
        a = bs.bs_eval_velocity(h)
        b = bs.bs_eval_velocity(h, serial=True)
        assert np.array_equal(a, b)
    bs.bs_mesh_free(h)


def test_pure_ray_tracing_convergence():
    """The paper's method alone (every pair ray traced) on the GPU: error
    against the analytic velocity of a smooth vortex under refinement
    (Section 3.2, Figure 4: about second order), on jittered Kuhn meshes of
    [-2, 2]^3, 24 x 24 lines; every node with 0.3 sigma < |x| < 1.6 sigma is
    compared.  At the coarsest mesh the GPU also matches the oracle."""
    claims = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_claims.json")))
    paper_p = claims["convergence_under_refinement"]["exponent"]
    L, sig = 2.0, 0.5
    hs, errs, errs_h = [], [], []
    for cells in (16, 24, 32, 48):
        xyz, tets, hh, b = W.kuhn_grid((-L,) * 3, (L,) * 3, (cells,) * 3)
        xyz = W.jitter_interior(xyz, b, hh, 0.1, 11)
        tets = W.orient_positive(xyz, tets)
        om, v = R.gaussian_vortex(xyz, sig)
        vg, st = gpu_eval((xyz, om, tets), kind=bs.BS_POLICY_PURE_RT, n_phi=24, n_theta=24)
        vh, sth = gpu_eval((xyz, om, tets), kind=bs.BS_POLICY_FIXED, n_phi=24, n_theta=24)
        r = np.linalg.norm(xyz, axis=1)
        sel = np.nonzero((r < 1.6 * sig) & (r > 0.3 * sig))[0]
        err = np.sqrt(np.sum((vg[sel] - v[sel]) ** 2) / np.sum(v[sel] ** 2))
        err_h = np.sqrt(np.sum((vh[sel] - v[sel]) ** 2) / np.sum(v[sel] ** 2))
        _say(f"{cells}^3 cells (h {hh[0]:.4f}, {xyz.shape[0]} nodes): pure RT rel error {err:.3e} "
             f"({st['t_eval_s'] * 1e3:.1f} ms), hybrid {err_h:.3e} ({sth['t_eval_s'] * 1e3:.1f} ms)")
        hs.append(hh[0])
        errs.append(err)
        errs_h.append(err_h)
        if cells == 16:
            tg = np.random.default_rng(0).choice(sel, size=16, replace=False)
            ref = oracle.evaluate(xyz, om, tets, oracle.make_policy("pure_rt", n_phi=24, n_theta=24), targets=tg)
            check(vg[tg], ref, "16^3 sample")
    p = np.polyfit(np.log(hs), np.log(errs), 1)[0]
    ph = np.polyfit(np.log(hs), np.log(errs_h), 1)[0]
    _say(f"fitted order: pure ray tracing {p:.2f}, hybrid (fixed rule) {ph:.2f} (the paper's fit: {paper_p})")
    assert 1.5 < p < 2.8
    assert abs(p - paper_p) < 0.7
    # the hybrid's far field starts at a cut proportional to h, which could
    # cost an order (the centroid rule's error summed over the far shells);
    # it is reported beside pure ray tracing and must still converge
    assert 1.0 < ph < 2.8


def test_hill_vortex_convergence():
    """The paper's test problem (Section 3.1, Table 1: Hill's spherical
    vortex, omega_theta = A r inside the unit sphere) on jittered Kuhn meshes
    of the ball whose boundary nodes lie on the sphere: pure ray tracing and
    the hybrid fixed rule at 16 x 16 lines against the closed form at every
    node inside 0.6 of the radius; both converge about second order.  At the
    coarsest mesh both match the oracle."""
    hs, errs, errs_h = [], [], []
    for cells in (10, 14, 20, 28):
        x, tets, _ = W.sphere_ball_mesh(cells=cells)
        om = R.hill_vorticity(x * (1.0 - 1e-12))
        sel = np.nonzero(np.linalg.norm(x, axis=1) < 0.6)[0]
        ref = R.hill_velocity(x[sel])
        vp, st = gpu_eval((x, om, tets), kind=bs.BS_POLICY_PURE_RT)
        vh, sth = gpu_eval((x, om, tets), kind=bs.BS_POLICY_FIXED)
        e_p = float(np.linalg.norm(vp[sel] - ref) / np.linalg.norm(ref))
        e_h = float(np.linalg.norm(vh[sel] - ref) / np.linalg.norm(ref))
        _say(f"Hill's vortex, {cells}^3 cells ({x.shape[0]} nodes, {tets.shape[0]} tets): rel error pure RT {e_p:.3e} "
             f"({st['t_eval_s'] * 1e3:.1f} ms), hybrid {e_h:.3e} ({sth['t_eval_s'] * 1e3:.1f} ms)")
        hs.append(2.0 / cells)
        errs.append(e_p)
        errs_h.append(e_h)
        if cells == 10:
            tg = np.random.default_rng(4).choice(sel, size=24, replace=False)
            check(vp[tg], oracle.evaluate(x, om, tets, oracle.make_policy("pure_rt"), targets=tg), "pure RT sample")
            check(vh[tg], oracle.evaluate(x, om, tets, oracle.make_policy("fixed"), targets=tg), "hybrid sample")
    p = np.polyfit(np.log(hs), np.log(errs), 1)[0]
    ph = np.polyfit(np.log(hs), np.log(errs_h), 1)[0]
    _say(f"Hill's vortex fitted order: pure ray tracing {p:.2f}, hybrid {ph:.2f}")
    assert 1.5 < p < 2.8 and 1.5 < ph < 2.8
    assert errs[-1] < 3e-3 and errs_h[-1] < 3e-3


@pytest.mark.parametrize("kind", ["fixed", "pure_rt"])
def test_off_node_points(kind):
    """Velocities at points that are not mesh nodes (Section 3.1 evaluates
    there): seeded points inside the mesh (inside tets), near nodes, and
    outside the mesh.  The oracle takes them as extra nodes that no tet has
    as a vertex.  The nodes' own evaluation is unchanged by the points."""
    m = W.make_config("C1")
    rng = np.random.default_rng(7)
    inside = rng.uniform(-0.97, 0.97, size=(150, 3))
    near = m.xyz[rng.choice(m.n_nodes, 20, replace=False)] + rng.normal(scale=1e-3, size=(20, 3))
    outside = rng.uniform(-1.0, 1.0, size=(30, 3))
    outside[:, 0] = np.sign(rng.uniform(-1, 1, 30)) * rng.uniform(1.05, 1.6, 30)
    pts = np.concatenate([inside, near, outside])
    pol = dict(kind=bs.BS_POLICY_FIXED) if kind == "fixed" else dict(kind=bs.BS_POLICY_PURE_RT)
    _say(f"off-node points, {kind}: {len(pts)} points")
    h = bs.bs_mesh_upload(m.xyz, m.omega, m.tets)
    bs.bs_set_policy(h, **pol)
    v_nodes = bs.bs_eval_velocity(h)
    vp, st = bs.bs_eval_points(h, pts, stats=True)
    v_nodes2 = bs.bs_eval_velocity(h)
    empty = bs.bs_eval_points(h, np.zeros((0, 3)))
    bs.bs_mesh_free(h)
    assert st["pairs"] == len(pts) * m.n_tets
    assert empty.shape == (0, 3)
    assert np.allclose(v_nodes2, v_nodes, rtol=0, atol=1e-14 * np.abs(v_nodes).max())
    xyz = np.concatenate([m.xyz, pts])
    om = np.concatenate([m.omega, np.zeros_like(pts)])
    tg = np.arange(m.n_nodes, m.n_nodes + len(pts))
    ref = oracle.evaluate(xyz, om, m.tets, oracle.make_policy(kind), targets=tg)
    check(vp, ref, "points")
