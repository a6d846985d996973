"""Host side of the Lagrangian driver: the re-tetrahedralisation of moved
nodes (Qhull Delaunay, standing in for the paper's external mesher) gives
positively oriented, non-flat tetrahedra that fill the points' convex hull
and use every point, also for the co-spherical points of a lattice."""
import numpy as np
from scipy.spatial import ConvexHull

import workloads as W
from paper_0712_1695_amd.lagrangian import retetrahedralise


def _check(xyz, tets):
    X = xyz[tets]
    det = np.linalg.det(X[:, 1:, :] - X[:, :1, :])
    edge = np.max(np.linalg.norm(X[:, :, None, :] - X[:, None, :, :], axis=-1).reshape(len(tets), -1), axis=1)
    assert np.all(det > 1e-6 * edge ** 3)
    hull = ConvexHull(xyz).volume
    assert abs(det.sum() / 6.0 - hull) <= 1e-10 * hull
    assert np.array_equal(np.unique(tets), np.arange(xyz.shape[0]))


def test_retetrahedralise_lattice_and_jittered_points():
    lo, hi = np.array([-1.0, -1.0, -0.5]), np.array([1.0, 1.0, 0.5])
    xyz, tets, h, b = W.kuhn_grid(lo, hi, (5, 5, 3))
    _check(xyz, retetrahedralise(xyz))  # co-spherical lattice: Qhull's flat tets dropped
    xj = W.jitter_interior(xyz, b, h, 0.3, 5)
    _check(xj, retetrahedralise(xj))
    rng = np.random.default_rng(6)
    pts = rng.uniform(-1.0, 1.0, (300, 3))
    _check(pts, retetrahedralise(pts))
