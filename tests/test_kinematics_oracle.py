"""Pins of the oracle's Lagrangian kinematics (oracle/kinematics.py) against
things other than its own formulas: exactness on globally linear velocity
fields, the divergence theorem on the star of every node (the volume-weighted
sum of the tetrahedra's gradients equals a surface integral over the star's
boundary, which never forms a gradient), and the Taylor polynomial of Heun's
method on a linear system."""
import numpy as np

import oracle.kinematics as K
import workloads as W


def _mesh(cells=(4, 3, 5), alpha=0.25, seed=3):
    lo, hi = np.array([-1.0, -0.5, -1.2]), np.array([1.0, 0.7, 0.9])
    xyz, tets, h, b = W.kuhn_grid(lo, hi, cells)
    xyz = W.jitter_interior(xyz, b, h, alpha, seed)
    return xyz, W.orient_positive(xyz, tets)


def test_linear_field_gradient_is_exact():
    """A globally linear velocity v = A x + c is its own interpolant: every
    tetrahedron's gradient, and so every node's mean, is A (not A^T)."""
    xyz, tets = _mesh()
    rng = np.random.default_rng(0)
    A = rng.standard_normal((3, 3))
    c = rng.standard_normal(3)
    v = xyz @ A.T + c
    G, vol = K.tet_gradients(xyz, tets, v)
    assert np.max(np.abs(G - A)) < 1e-12
    assert np.all(vol > 0)
    g = K.nodal_velocity_gradient(xyz, tets, v)
    assert np.max(np.abs(g - A)) < 1e-12
    s = K.stretching(g, xyz)  # any vorticity: (w . grad) v = A w
    assert np.max(np.abs(s - xyz @ A.T)) < 1e-12


def _star_surface_integrals(xyz, tets, v, node):
    """(sum over the boundary faces of the node's star of int v n^T dS,
    (1/3) sum of int x . n dS): both exact for linear integrands by the
    face-centroid rule, both from face normals alone."""
    star = np.nonzero(np.any(tets == node, axis=1))[0]
    faces = {}
    for t in star:
        for f in range(4):
            tri = tuple(sorted(int(k) for j, k in enumerate(tets[t]) if j != f))
            faces.setdefault(tri, []).append((t, int(tets[t][f])))
    flux = np.zeros((3, 3))
    vol3 = 0.0
    for tri, owners in faces.items():
        if len(owners) != 1:  # shared by two tets of the star: interior face
            continue
        opp = owners[0][1]
        p = xyz[list(tri)]
        n = 0.5 * np.cross(p[1] - p[0], p[2] - p[0])  # area-weighted normal
        if np.dot(n, xyz[opp] - p[0]) > 0:
            n = -n  # outward from the star (away from the opposite vertex)
        vbar = v[list(tri)].mean(axis=0)
        flux += np.outer(vbar, n)
        vol3 += np.dot(p.mean(axis=0), n)
    return flux, vol3 / 3.0


def test_star_sums_match_divergence_theorem():
    """For a continuous piecewise-linear v, sum_T |T| grad v_T over the
    node's star equals the boundary integral of v n^T, and the star's volume
    equals (1/3) of the boundary integral of x . n; so the node's mean
    gradient times that volume must equal the boundary flux, at interior and
    boundary nodes alike."""
    xyz, tets = _mesh()
    rng = np.random.default_rng(1)
    v = rng.standard_normal(xyz.shape)
    g = K.nodal_velocity_gradient(xyz, tets, v)
    for node in rng.choice(xyz.shape[0], 25, replace=False):
        flux, vol = _star_surface_integrals(xyz, tets, v, node)
        assert vol > 0
        assert np.max(np.abs(g[node] * vol - flux)) < 1e-12 * max(1.0, np.max(np.abs(flux)))


def test_unreferenced_node_gets_zero():
    xyz, tets = _mesh(cells=(2, 2, 2))
    xyz = np.vstack([xyz, [[5.0, 5.0, 5.0]]])
    v = np.random.default_rng(2).standard_normal(xyz.shape)
    g = K.nodal_velocity_gradient(xyz, tets, v)
    assert np.all(g[-1] == 0.0)


def test_heun_is_second_order_taylor_on_linear_system():
    """Heun's method on y' = B y advances by I + dt B + dt^2 B^2 / 2 exactly."""
    rng = np.random.default_rng(4)
    B = rng.standard_normal((3, 3))
    C = rng.standard_normal((3, 3))
    x0, w0 = rng.standard_normal((7, 3)), rng.standard_normal((7, 3))
    dt = 0.13
    x1, w1 = K.heun((x0, w0), lambda y: (y[0] @ B.T, y[1] @ C.T), dt)
    PB = np.eye(3) + dt * B + 0.5 * dt * dt * B @ B
    PC = np.eye(3) + dt * C + 0.5 * dt * dt * C @ C
    assert np.max(np.abs(x1 - x0 @ PB.T)) < 1e-14
    assert np.max(np.abs(w1 - w0 @ PC.T)) < 1e-14
