"""Pins of the FP64 oracle against things other than itself: a library
Gauss-Legendre routine, closed-form simplex moments, closed-form
velocities (uniform vorticity in a ball and in a box), analytic line
integrals through a box (uniform and globally linear vorticity), brute-force
integration of single tetrahedra by two independent routes, invariances
(precheck on/off, linearity, superposition over a tet partition, reflection
equivariance) and second-order convergence under refinement.

Each test names the passage of the paper it checks."""
import json
import math
import os

import numpy as np
import pytest

import oracle as O
import oracle.references as R
import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
BOX_LO = np.array([-1.0, -1.0, -1.0])
BOX_HI = np.array([1.0, 1.0, 1.0])


def _cube_mesh(cells=4, alpha=0.2, seed=1):
    xyz, tets, h, b = W.kuhn_grid(BOX_LO, BOX_HI, (cells,) * 3)
    xyz = W.jitter_interior(xyz, b, h, alpha, seed)
    return xyz, W.orient_positive(xyz, tets), b


# --------------------------------------------------------------- eq. 3 tables

@pytest.mark.parametrize("n", [1, 2, 3, 4, 7, 16, 33, 64])
def test_gauss_legendre_matches_library(n):
    """Section 2, eq. 3: N-point Gauss-Legendre nodes and weights."""
    t, w = O.gauss_legendre(n)
    tr, wr = np.polynomial.legendre.leggauss(n)
    assert np.max(np.abs(t - tr)) < 1e-14
    assert np.max(np.abs(w - wr)) < 1e-14


@pytest.mark.parametrize("n", [2, 5, 16])
def test_gauss_legendre_polynomial_exactness(n):
    t, w = O.gauss_legendre(n)
    for k in range(2 * n):
        exact = 0.0 if k % 2 else 2.0 / (k + 1)
        assert abs(np.sum(w * t ** k) - exact) < 1e-13
    k = 2 * n
    assert abs(np.sum(w * t ** k) - 2.0 / (k + 1)) > 1e-11  # degree is exactly 2n-1


@pytest.mark.parametrize("n", [4, 8, 16, 32])
def test_half_sphere_measure(n):
    """Section 2.2 item 3: the factors k_nm integrate the half sphere of line
    directions with the 1/(4 pi) of eq. 1, so they sum to 1/2 as N grows.
    At N = 4 the sum is the 4-point Gauss value of
    (pi/16) * 2 * integral of sin((1+t) pi/2) dt over [-1, 1]."""
    s, k = O.angular_tables(n, n)
    tr, wr = np.polynomial.legendre.leggauss(n)
    expect = math.pi / 16.0 * 2.0 * np.sum(wr * np.sin((1.0 + tr) * math.pi / 2.0))
    assert abs(k.sum() - expect) < 1e-14
    assert abs(k.sum() - 0.5) < (1e-5 if n == 4 else 1e-13)
    # unit directions covering the half sphere s_y > 0
    assert np.allclose(np.linalg.norm(s, axis=1), 1.0, atol=1e-15)
    assert np.all(s[:, 1] > 0)


# --------------------------------------------------------------- tet rules

@pytest.mark.parametrize("k,degree", [(1, 1), (4, 2), (11, 4)])
def test_tet_rule_exactness(k, degree):
    """Far-field Gauss rules (Introduction): symmetric 1/4/11-point rules are
    exact for every barycentric monomial up to their degree, not beyond."""
    lam, w = O.tet_rule(k)
    assert abs(w.sum() - 1.0) < 1e-15
    assert np.allclose(lam.sum(axis=1), 1.0, atol=1e-15)
    exps = [e for e in np.ndindex(degree + 2, degree + 2, degree + 2, degree + 2)]
    worst_in, worst_out = 0.0, 0.0
    for e in exps:
        d = sum(e)
        if d > degree + 1:
            continue
        approx = float(np.sum(w * np.prod(lam ** np.array(e)[None, :], axis=1)))
        err = abs(approx - R.simplex_moment(e))
        if d <= degree:
            worst_in = max(worst_in, err)
        else:
            worst_out = max(worst_out, err)
    assert worst_in < 1e-15 * 50
    assert worst_out > 1e-6


# --------------------------------------------------------------- closed forms

def test_uniform_ball_closed_form():
    """Section 2, eqs. 2-3 with the sign of R restored and the pi/16
    constant: the angular rule applied to the exact chords of a ball with
    uniform vorticity reproduces v = omega x x / 3 (spectral convergence,
    the angular integrand is a polynomial in s)."""
    x = np.array([0.3, -0.2, 0.4])
    w0 = np.array([0.7, -0.3, 0.5])
    ref = R.ball_uniform_velocity(x, w0)
    errs = []
    for n in (2, 4, 8, 16):
        s, k = O.angular_tables(n, n)
        errs.append(np.max(np.abs(R.ball_line_sum(s, k, x, w0) - ref)) / np.max(np.abs(ref)))
    assert errs[-1] < 1e-14
    assert errs[0] > errs[1] > errs[2] > errs[3]


def test_box_closed_form_against_brute_force_sum():
    """The box closed form (surface potential of a rectangle) against the sum
    of exact single-tetrahedron velocities over a tet mesh of the box."""
    xyz, tets, _ = _cube_mesh(cells=2, alpha=0.15, seed=5)
    w0 = np.array([0.4, 0.9, -0.6])
    for x in (np.array([0.13, -0.21, 0.05]), np.array([0.9, 0.8, -0.7])):
        tot = np.zeros(3)
        for t in tets:
            tot += R.tet_cone_brute_force(x, xyz[t], np.tile(w0, (4, 1)), order=80)
        ref = R.box_uniform_velocity(x, BOX_LO, BOX_HI, w0)
        assert np.max(np.abs(tot - ref)) < 1e-11 * np.max(np.abs(ref))


@pytest.mark.parametrize("linear", [False, True])
def test_mesh_chords_sum_to_box_line_integrals(linear):
    """Section 2.1, eqs. 4-5: on any tetrahedral mesh of a box the per-tet
    chord integrals (Moller-Trumbore hits, area-coordinate vorticity, exact
    trapezoid, incident tets from the node to the opposite face) add up, line
    by line, to the exact line integral through the box, so pure ray tracing
    equals the analytic line sum to rounding for uniform and for globally
    linear vorticity.  Targets include interior, face, edge and corner nodes."""
    xyz, tets, bnd = _cube_mesh(cells=4, alpha=0.2, seed=1)
    w0 = np.array([0.7, -0.3, 0.5])
    G = np.array([[0.2, -0.5, 0.1], [0.3, 0.1, -0.4], [-0.2, 0.6, 0.3]]) if linear else np.zeros((3, 3))
    om = W.field_linear(xyz, w0, G)
    targets = np.array([0, 2, 10, 31, 62, 93, 124])
    for N, M in ((8, 12), (16, 16)):
        v = O.evaluate(xyz, om, tets, O.make_policy("pure_rt", n_phi=N, n_theta=M), targets=targets)
        s, k = O.angular_tables(N, M)
        for i, ti in enumerate(targets):
            ref = R.cube_line_sum(s, k, xyz[ti], BOX_LO, BOX_HI, w0, G)
            assert np.max(np.abs(v[i] - ref)) < 1e-13, (N, M, ti)


def test_box_uniform_converges_to_closed_form():
    """Section 3.2: accuracy controlled by the quadrature order.  Pure ray
    tracing of uniform vorticity on a box mesh converges to the Biot-Savart
    closed form as N = M grows."""
    xyz, tets, _ = _cube_mesh(cells=4, alpha=0.2, seed=1)
    w0 = np.array([0.7, -0.3, 0.5])
    om = W.field_uniform(xyz, w0)
    targets = np.array([31, 62, 93])
    errs = []
    for n in (8, 16, 32, 64):
        v = O.evaluate(xyz, om, tets, O.make_policy("pure_rt", n_phi=n, n_theta=n), targets=targets)
        ref = np.array([R.box_uniform_velocity(xyz[t], BOX_LO, BOX_HI, w0) for t in targets])
        errs.append(np.max(np.abs(v - ref)) / np.max(np.abs(ref)))
    assert errs[1] < 2e-2 and errs[3] < 1e-3
    assert errs[0] > errs[1] > errs[2] > errs[3]


# --------------------------------------------------------------- single tets

def test_brute_force_references_agree():
    """Two independent exact references (signed face cones with an exact
    radial integral; 8-way subdivision with a degree-4 rule) agree."""
    m = W.single_tet(3)
    tv, tw = m.xyz[m.tets[0]], m.omega[m.tets[0]]
    for x in ([2.0, 1.5, -1.0], [0.9, 0.8, 0.7], [0.3, 0.3, -0.4]):
        a = R.tet_cone_brute_force(x, tv, tw, order=48)
        b = R.tet_subdivision(x, tv, tw, levels=4)
        assert np.max(np.abs(a - b)) < 2e-9 * np.max(np.abs(a))


def test_gauss_rules_against_brute_force():
    """Far-field rules: error shrinks with the rule's degree and with
    distance, and the sign and 1/(4 pi) factor match the exact integral."""
    m = W.single_tet(4)
    tv, tw = m.xyz[m.tets[0]], m.omega[m.tets[0]]
    for x, tol in (([3.0, 2.5, -2.0], (0.2, 2e-3, 5e-5)), ([6.0, -5.0, 4.0], (0.05, 1e-3, 5e-6))):
        ref = R.tet_cone_brute_force(x, tv, tw, order=40)
        errs = [np.max(np.abs(O.pair(x, tv, tw, r) - ref)) / np.max(np.abs(ref)) for r in (0, 1, 2)]
        assert errs[0] < tol[0] and errs[1] < tol[1] and errs[2] < tol[2], errs
        assert errs[0] > errs[1] > errs[2]


def test_ray_tracing_single_tet_converges():
    """Section 2.1: ray tracing of one tetrahedron converges to its exact
    velocity as the angular rule is refined, for a distant target, a close
    target and a target at one of its vertices (incident case)."""
    m = W.single_tet(3)
    tv, tw = m.xyz[m.tets[0]], m.omega[m.tets[0]]
    for x in ([0.9, 0.8, 0.7], [0.3, 0.3, -0.4]):
        ref = R.tet_cone_brute_force(x, tv, tw, order=48)
        errs = [np.max(np.abs(O.pair(x, tv, tw, 3, N=n, M=n) - ref)) / np.max(np.abs(ref)) for n in (32, 128, 256)]
        assert errs[2] < 1e-3 and errs[0] > errs[2]
    ids = [5, 6, 7, 8]
    for j in range(4):
        x = tv[j]
        ref = R.tet_cone_brute_force(x, tv, tw, order=64)
        errs = [np.max(np.abs(O.pair(x, tv, tw, 3, N=n, M=n, self_index=ids[j], ids=ids, omega_x=tw[j]) - ref))
                / np.max(np.abs(ref)) for n in (16, 64, 256)]
        assert errs[2] < 2e-2 and errs[2] < 0.2 * errs[0], (j, errs)


def test_precheck_never_changes_results():
    """Section 2.1 precheck: skipping lines with (r.s)^2 < |r|^2 - 2h^2 is
    conservative (the tet lies in the ball of radius h about any vertex), so
    results are bitwise identical with and without it."""
    m = W.make_config("C1", scale=(5, 5, 5))
    targets = np.arange(0, m.n_nodes, 3)
    a = O.evaluate(m.xyz, m.omega, m.tets, O.make_policy("pure_rt", precheck=True), targets=targets)
    b = O.evaluate(m.xyz, m.omega, m.tets, O.make_policy("pure_rt", precheck=False), targets=targets)
    assert np.array_equal(a, b)


# --------------------------------------------------------------- invariances

def test_linearity_and_partition_superposition():
    """Eq. 1 is linear in omega, and Section 2.2: splitting the tets among
    processors and summing the partial velocities gives the full result."""
    m = W.make_config("C1", scale=(5, 5, 5))
    rng = np.random.default_rng(0)
    om2 = rng.standard_normal(m.omega.shape)
    targets = np.arange(0, m.n_nodes, 5)
    pol = O.make_policy("fixed")
    v1, rules = O.evaluate(m.xyz, m.omega, m.tets, pol, targets=targets, return_rules=True)
    v2 = O.evaluate(m.xyz, om2, m.tets, pol, targets=targets)
    v12 = O.evaluate(m.xyz, 2.0 * m.omega - 3.0 * om2, m.tets, pol, targets=targets)
    assert np.max(np.abs(v12 - (2 * v1 - 3 * v2))) < 1e-13 * np.max(np.abs(v12))
    part = rng.random(m.n_tets) < 0.4
    va = O.evaluate(m.xyz, m.omega, m.tets[part], targets=targets, pair_rules=rules[:, part])
    vb = O.evaluate(m.xyz, m.omega, m.tets[~part], targets=targets, pair_rules=rules[:, ~part])
    assert np.max(np.abs(va + vb - v1)) < 1e-13 * np.max(np.abs(v1))


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_axis_reflection_equivariance(axis):
    """The Gauss nodes are symmetric, so reflecting the mesh in a coordinate
    plane maps the line set onto itself; with omega transformed as an axial
    vector the velocity reflects exactly (up to rounding)."""
    m = W.make_config("C1", scale=(4, 4, 4))
    S = np.eye(3)
    S[axis, axis] = -1.0
    xyz2 = m.xyz @ S
    om2 = -(m.omega @ S)  # det(S) * S omega
    tets2 = W.orient_positive(xyz2, m.tets)
    targets = np.arange(0, m.n_nodes, 4)
    pol = O.make_policy("pure_rt", n_phi=8, n_theta=8)
    v = O.evaluate(m.xyz, m.omega, m.tets, pol, targets=targets)
    v2 = O.evaluate(xyz2, om2, tets2, pol, targets=targets)
    assert np.max(np.abs(v2 - v @ S)) < 1e-13 * np.max(np.abs(v))


@pytest.mark.slow
def test_second_order_convergence():
    """Section 3.2 (Figure 4): with the angular error below the resolution
    error, pure ray tracing converges about second order in h.  Smooth,
    divergence-free vorticity with an analytic velocity on jittered Kuhn
    meshes of [-2, 2]^3."""
    claims = json.load(open(os.path.join(GOLDEN, "paper_claims.json")))
    paper_p = claims["convergence_under_refinement"]["exponent"]
    L, sig = 2.0, 0.5
    hs, errs = [], []
    for cells in (24, 32, 48):
        xyz, tets, h, b = W.kuhn_grid((-L,) * 3, (L,) * 3, (cells,) * 3)
        xyz = W.jitter_interior(xyz, b, h, 0.1, 11)
        tets = W.orient_positive(xyz, tets)
        om, v = R.gaussian_vortex(xyz, sig)
        r = np.linalg.norm(xyz, axis=1)
        cand = np.nonzero((r < 1.6 * sig) & (r > 0.3 * sig))[0]
        tg = np.random.default_rng(0).choice(cand, size=12, replace=False)
        vv = O.evaluate(xyz, om, tets, O.make_policy("pure_rt", n_phi=24, n_theta=24), targets=tg)
        errs.append(np.sqrt(np.mean(np.sum((vv - v[tg]) ** 2, axis=1)) / np.mean(np.sum(v[tg] ** 2, axis=1))))
        hs.append(h[0])
    p = np.polyfit(np.log(hs), np.log(errs), 1)[0]
    assert 1.5 < p < 2.8, (p, errs)
    assert abs(p - paper_p) < 0.7


# --------------------------------------------------------------- Hill's vortex

def test_hill_closed_form_is_the_velocity_of_its_vorticity():
    """Section 3.1's Hill's vortex, in the corrected form: inside the sphere
    the velocity's curl is A(-y, x, 0) and its divergence zero (central
    differences), and the velocity is continuous across |x| = a (the inner
    form against the outer dipole of a sphere moving at 2 A a^2 / 15)."""
    A, a, e = 1.7, 1.3, 1e-5
    rng = np.random.default_rng(5)
    pts = rng.uniform(-0.6, 0.6, size=(20, 3)) * a
    for p in pts:
        J = np.zeros((3, 3))
        for k in range(3):
            d = np.zeros(3)
            d[k] = e
            J[:, k] = (R.hill_velocity((p + d)[None], A, a)[0] - R.hill_velocity((p - d)[None], A, a)[0]) / (2 * e)
        curl = np.array([J[2, 1] - J[1, 2], J[0, 2] - J[2, 0], J[1, 0] - J[0, 1]])
        assert np.allclose(curl, A * np.array([-p[1], p[0], 0.0]), atol=1e-8)
        assert abs(np.trace(J)) < 1e-8
    # continuity across the sphere, and decay far away
    dirs = rng.standard_normal((30, 3))
    dirs /= np.linalg.norm(dirs, axis=1)[:, None]
    vin = R.hill_velocity(dirs * a * (1 - 1e-12), A, a)
    vout = R.hill_velocity(dirs * a * (1 + 1e-12), A, a)
    assert np.max(np.abs(vin - vout)) < 1e-9 * A * a * a
    far = R.hill_velocity(dirs * 50 * a, A, a)
    assert np.max(np.abs(far)) < 1e-5 * A * a * a
    # omega = A (-y, x, 0) inside, zero outside
    assert np.allclose(R.hill_vorticity(pts, A, a), A * np.stack([-pts[:, 1], pts[:, 0], 0 * pts[:, 0]], 1))
    assert np.all(R.hill_vorticity(dirs * 1.01 * a, A, a) == 0.0)


@pytest.mark.slow
def test_hill_vortex_pure_ray_tracing_converges():
    """The paper's test problem (Section 3.1, Table 1): Hill's vortex on a
    jittered Kuhn mesh of the ball (the cube carried onto the sphere), pure
    ray tracing with 16 x 16 lines, against the closed form at nodes inside
    0.6 a.  The linear vorticity is reproduced exactly inside the
    polyhedron, whose boundary nodes lie on the sphere, so the error falls
    about second order in h (the paper's 16 x 16 errors on its random point
    sets are of order 1e-2)."""
    errs = []
    for cells in (6, 10):
        x, tets, _ = W.sphere_ball_mesh(cells=cells)
        om = R.hill_vorticity(x * (1.0 - 1e-12))  # boundary nodes (on the sphere) carry the inner field
        tg = np.nonzero(np.linalg.norm(x, axis=1) < 0.6)[0]
        v = O.evaluate(x, om, tets, O.make_policy("pure_rt"), targets=tg)
        ref = R.hill_velocity(x[tg])
        errs.append(np.linalg.norm(v - ref) / np.linalg.norm(ref))
    assert errs[0] < 0.05, errs
    assert errs[1] < 0.55 * errs[0], errs  # (6/10)^2 = 0.36 for second order, 0.6 for first
