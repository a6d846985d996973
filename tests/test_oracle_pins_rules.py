"""Pins of the parts of the FP64 oracle that the parity tests only compare
against the GPU: the fixed distance rule (decided in binary32), the mean edge
length over unique edges, the ray-tracing branch for targets strictly inside
a tetrahedron, and the selector's pair features.  Each test checks the oracle
against values fixed independently of its code: exact binary32 distances one
unit in the last place either side of each cut, closed-form edge sums of an
unjittered Kuhn grid, the analytic line integrals through a box, and features
worked out by hand for a reference tetrahedron."""
import math

import numpy as np
import pytest

import oracle as O
import oracle.references as R
from oracle.features import pair_features
import workloads as W

RT, G11, G4, G1 = O.RULE_RT, O.RULE_G11, O.RULE_G4, O.RULE_G1

# a regular tetrahedron whose centroid is exactly the origin: every edge has
# length 2 sqrt(2), so the mean edge length is 2 sqrt(2)
REG_TET = np.array([[1.0, 1.0, 1.0], [1.0, -1.0, -1.0], [-1.0, 1.0, -1.0], [-1.0, -1.0, 1.0]])
HBAR_REG = 2.0 * math.sqrt(2.0)


def _f32_d2(dx, dy, dz):
    """Squared distance in binary32 in the reading's order:
    ((dx*dx + dy*dy) + dz*dz), every operation rounded."""
    f = np.float32
    sx, sy, sz = f(f(dx) * f(dx)), f(f(dy) * f(dy)), f(f(dz) * f(dz))
    return f(f(sx + sy) + sz)


def _offsets_hitting(target):
    """Binary32 offsets (a, b) with fl32(fl32(a*a) + fl32(b*b)) == target, for
    target and its two binary32 neighbours (found by a small search: a near
    sqrt(target), b a small multiple of a power of two)."""
    f = np.float32
    want = {f(np.nextafter(target, f(0))): None, f(target): None, f(np.nextafter(target, f(np.inf))): None}
    a0 = f(math.sqrt(float(target)))
    ulp_t = float(np.spacing(f(target)))
    e = math.floor(math.log2(ulp_t) / 2)
    a = a0
    for _ in range(48):
        a = np.nextafter(a, f(0))
    for _ in range(96):
        for j in range(0, 40):
            b = f(j * 2.0 ** e)
            d2 = _f32_d2(a, b, f(0))
            if d2 in want and want[d2] is None:
                want[d2] = (float(a), float(b))
        a = np.nextafter(a, f(np.inf))
    assert all(v is not None for v in want.values()), want
    return want


@pytest.mark.parametrize("cuts", [(2.0, 4.0, 8.0), (1.7, 3.3, 6.1)])
def test_fixed_rule_one_ulp_either_side_of_each_cut(cuts):
    """Distance rule (Introduction: Gauss rules for distant elements; ring
    workload: ray tracing within 2 mean edge lengths): with d the node to
    centroid distance, d < c_rt is ray traced, c_rt <= d < c_11 takes the
    11-point rule, c_11 <= d < c_4 the 4-point rule, beyond that the centroid
    rule.  The comparison is on binary32 squares, fl32((c h)^2), so a node
    whose binary32 d^2 is one unit in the last place below a cut takes the
    nearer rule, and one exactly at or above it the farther rule."""
    near, g11, g4 = cuts
    f = np.float32
    extra, expect = [], []
    for k, (cut, inner, outer) in enumerate(((near, RT, G11), (g11, G11, G4), (g4, G4, G1))):
        thr = f((cut * HBAR_REG) ** 2)
        for d2, (a, b) in sorted(_offsets_hitting(thr).items()):
            p = [0.0, 0.0, 0.0]
            p[k % 3] = a            # the offsets on different axes for each cut
            p[(k + 1) % 3] = b
            extra.append(p)
            expect.append(inner if d2 < thr else outer)
    # vertices: incident pairs are ray traced at any distance; a non-incident
    # node at a vertex's distance is not
    xyz = np.vstack([REG_TET, np.array(extra), -REG_TET[0:1]])
    om = np.tile([0.3, -0.2, 0.5], (xyz.shape[0], 1))
    tets = W.orient_positive(xyz, np.array([[0, 1, 2, 3]], dtype=np.int32))
    assert W.signed_volumes6(xyz, tets)[0] > 0
    targets = np.arange(4, xyz.shape[0] - 1)
    _, rules, cnt = O.evaluate(xyz, om, tets, O.make_policy("fixed", near_cut=near, d_g11=g11, d_g4=g4),
                               targets=targets, return_rules=True, return_counters=True)
    assert abs(cnt["hbar"] - HBAR_REG) < 1e-15 * HBAR_REG
    assert list(rules[:, 0]) == expect
    # tiny cuts: the vertices (distance sqrt(3) = 0.61 hbar) are beyond all
    # of them, yet incident; the node at -v0 is just as far and not incident
    pol = O.make_policy("fixed", near_cut=0.1, d_g11=0.2, d_g4=0.3)
    _, r2 = O.evaluate(xyz, om, tets, pol, targets=np.array([0, 1, 2, 3, xyz.shape[0] - 1]), return_rules=True)
    assert list(r2[:, 0]) == [RT, RT, RT, RT, G1]


def _kuhn_edge_closed_form(cells, lo, hi):
    """Unique edges of a Kuhn-split grid: every cell edge, one diagonal on
    every cell face, one body diagonal per cell.  Returns (count, length sum)."""
    nx, ny, nz = cells
    hx, hy, hz = [(hi[c] - lo[c]) / cells[c] for c in range(3)]
    groups = [
        (nx * (ny + 1) * (nz + 1), hx), ((nx + 1) * ny * (nz + 1), hy), ((nx + 1) * (ny + 1) * nz, hz),
        (nx * ny * (nz + 1), math.hypot(hx, hy)), (nx * (ny + 1) * nz, math.hypot(hx, hz)),
        ((nx + 1) * ny * nz, math.hypot(hy, hz)), (nx * ny * nz, math.sqrt(hx * hx + hy * hy + hz * hz)),
    ]
    return sum(c for c, _ in groups), sum(c * l for c, l in groups)


@pytest.mark.parametrize("cells", [(3, 4, 2), (1, 1, 1), (5, 2, 3)])
def test_mean_edge_is_the_mean_over_unique_edges(cells):
    """Ring workload's cut unit: the mean edge length is the mean over the
    mesh's unique edges (an edge shared by many tetrahedra counts once).  On
    an unjittered Kuhn grid with unequal spacings it equals the closed-form
    sum over axis edges, face diagonals and body diagonals divided by their
    count, whatever the order of the tetrahedra and of their vertices."""
    lo, hi = (0.0, -0.5, 0.25), (1.5, 0.5, 0.95)
    xyz, tets, _, _ = W.kuhn_grid(lo, hi, cells)
    count, total = _kuhn_edge_closed_form(cells, lo, hi)
    exact = total / count
    assert abs(O.mean_edge(xyz, tets) - exact) < 1e-14 * exact
    rng = np.random.default_rng(0)
    shuffled = tets[rng.permutation(tets.shape[0])]
    shuffled = np.take_along_axis(shuffled, np.argsort(rng.random(shuffled.shape), axis=1), axis=1)
    assert abs(O.mean_edge(xyz, shuffled) - exact) < 1e-14 * exact
    # the mean over edge instances (6 per tetrahedron) is a different number,
    # so the closed form tells the two readings apart
    e = xyz[tets[:, [1, 2, 3, 2, 3, 3]]] - xyz[tets[:, [0, 0, 0, 1, 1, 2]]]
    assert abs(np.linalg.norm(e, axis=2).mean() - exact) > 1e-3 * exact


@pytest.mark.parametrize("linear", [False, True])
def test_targets_strictly_inside_tets_match_box_line_integrals(linear):
    """Section 2.1, eq. 5 with the sign of R, for evaluation points that are
    not nodes (Section 3's random points): the line through a point strictly
    inside a tetrahedron enters behind the point and leaves in front of it,
    and the chord is split at R = 0 with the vorticity there.  The per-tet
    chords then still add up to the exact line integral through the box, for
    uniform and for globally linear vorticity."""
    lo, hi = np.array([-1.0, -1.0, -1.0]), np.array([1.0, 1.0, 1.0])
    xyz, tets, h, b = W.kuhn_grid(lo, hi, (4, 4, 4))
    xyz = W.jitter_interior(xyz, b, h, 0.2, 1)
    tets = W.orient_positive(xyz, tets)
    lams = np.array([[0.1, 0.2, 0.3, 0.4], [0.25, 0.25, 0.25, 0.25], [0.05, 0.05, 0.45, 0.45],
                     [0.7, 0.1, 0.1, 0.1], [0.02, 0.9, 0.03, 0.05]])
    pick = np.random.default_rng(3).choice(tets.shape[0], size=lams.shape[0], replace=False)
    pts = np.einsum("kj,kjc->kc", lams, xyz[tets[pick]])
    allx = np.vstack([xyz, pts])  # unreferenced nodes: no tetrahedron has them as a vertex
    w0 = np.array([0.7, -0.3, 0.5])
    G = np.array([[0.2, -0.5, 0.1], [0.3, 0.1, -0.4], [-0.2, 0.6, 0.3]]) if linear else np.zeros((3, 3))
    om = W.field_linear(allx, w0, G)
    targets = np.arange(xyz.shape[0], allx.shape[0])
    for N, M in ((8, 12), (16, 16)):
        v = O.evaluate(allx, om, tets, O.make_policy("pure_rt", n_phi=N, n_theta=M), targets=targets)
        s, k = O.angular_tables(N, M)
        for i, ti in enumerate(targets):
            ref = R.cube_line_sum(s, k, allx[ti], lo, hi, w0, G)
            assert np.max(np.abs(v[i] - ref)) < 1e-13 * max(1.0, np.max(np.abs(ref))), (N, M, i)


def test_pair_features_hand_computed():
    """The selector's 16 features (distance and edge ratios, barycentric
    direction, face angles with outward normals, incidence, shape, plane
    distance, constant) of the unit corner tetrahedron, worked out by hand,
    for a node off the element and for one of its vertices, in two vertex
    orders (the outward normals must not depend on the order)."""
    tv = np.array([[0.0, 0.0, 0.0], [1.0, 0.0, 0.0], [0.0, 1.0, 0.0], [0.0, 0.0, 1.0]])
    hbar = 0.5
    r3, r2 = math.sqrt(3.0), math.sqrt(2.0)
    # node x = (1, 1, 1): c = centroid - x = -(3/4)(1, 1, 1), d = 3 sqrt3 / 4,
    # h_T = sqrt2, h_min = 1, lambda = (-2, 1, 1, 1), outward normals
    # (1,1,1)/sqrt3 and -e_x, -e_y, -e_z, plane distances 2/sqrt3, 1, 1, 1
    d = 0.75 * r3
    k = r2 / d
    off = [d / r2, d / hbar, r2, hbar / d, k, k, k, -2 * k, 1.0, -1 / r3, -1 / r3, -1 / r3, 0.0,
           1 / (2 * r2), 1 / r2, 1.0]
    # vertex x = v0 (incident): d = sqrt3 / 4, lambda = (1, 0, 0, 0), the
    # direction to the centroid reversed gives cosines -1 and 1/sqrt3 (x3),
    # x lies on three face planes
    d0 = 0.25 * r3
    on = [d0 / r2, d0 / hbar, r2, hbar / d0, r2 / d0, 0.0, 0.0, 0.0, 1 / r3, 1 / r3, 1 / r3, -1.0, 1.0,
          1 / (2 * r2), 0.0, 1.0]
    for order in ([0, 1, 2, 3], [2, 0, 3, 1]):
        t = tv[order]
        assert np.allclose(pair_features([1.0, 1.0, 1.0], t, hbar), off, rtol=0, atol=1e-14)
        assert np.allclose(pair_features(tv[0], t, hbar, incident=True), on, rtol=0, atol=1e-14)
