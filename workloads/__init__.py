"""Seeded synthetic inputs: Kuhn-split tetrahedral grids, node jitter and
nodal vorticity fields.

This module only builds inputs (node coordinates, connectivity, nodal
vorticity).  It holds none of the velocity method's arithmetic, so both the
GPU library and the CPU oracle can be fed from it.

The paper evaluates the velocity at the nodes of a tetrahedralised point
set carrying a piecewise-linear vorticity (Section 2).  Its own point sets
(random points in a sphere, TetGen meshes, Gaussian-ring stations) are not
available, so the workloads here are structured grids, each hexahedral cell
split into six tetrahedra around its main diagonal (Kuhn / Freudenthal
split, which is conforming across cells), with the interior nodes jittered
by a seeded uniform perturbation.
"""
from __future__ import annotations

import dataclasses
import itertools
from typing import Callable, Dict, Optional, Tuple

import numpy as np

__all__ = [
    "Mesh",
    "kuhn_grid",
    "jitter_interior",
    "orient_positive",
    "signed_volumes6",
    "field_gaussian_swirl",
    "field_ring",
    "field_rings",
    "field_fourier_curl",
    "field_uniform",
    "field_linear",
    "make_config",
    "CONFIGS",
    "single_tet",
    "ball_mesh",
    "sphere_ball_mesh",
]


@dataclasses.dataclass
class Mesh:
    """A tetrahedral mesh with nodal vorticity.

    xyz:   float64 [n, 3] node coordinates
    omega: float64 [n, 3] nodal vorticity (linear inside each tetrahedron)
    tets:  int32   [T, 4] node indices per tetrahedron
    h:     float64 [3]    grid spacing per axis (structured grids only)
    name:  str            workload label
    """

    xyz: np.ndarray
    omega: np.ndarray
    tets: np.ndarray
    h: np.ndarray
    name: str = ""
    boundary: Optional[np.ndarray] = None

    @property
    def n_nodes(self) -> int:
        return int(self.xyz.shape[0])

    @property
    def n_tets(self) -> int:
        return int(self.tets.shape[0])


def _node_id(i, j, k, nx, ny):
    return i + (nx + 1) * (j + (ny + 1) * k)


def kuhn_grid(lo, hi, cells) -> Tuple[np.ndarray, np.ndarray, np.ndarray, np.ndarray]:
    """Nodes and tetrahedra of a box split into nx*ny*nz cells, six tets each.

    Each cell's six tetrahedra follow the monotone lattice paths from the
    cell's (0,0,0) corner to its (1,1,1) corner, one per permutation of the
    axes.  Every cell uses the same split, so shared faces match.

    Returns (xyz [n,3] f64, tets [T,4] i32, h [3] f64, boundary [n] bool).
    """
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    nx, ny, nz = (int(c) for c in cells)
    h = (hi - lo) / np.array([nx, ny, nz], dtype=np.float64)
    ii, jj, kk = np.meshgrid(np.arange(nx + 1), np.arange(ny + 1), np.arange(nz + 1), indexing="ij")
    # node id = i + (nx+1)*(j + (ny+1)*k): flatten in k-major order
    ii = ii.transpose(2, 1, 0).ravel()
    jj = jj.transpose(2, 1, 0).ravel()
    kk = kk.transpose(2, 1, 0).ravel()
    xyz = np.stack([lo[0] + ii * h[0], lo[1] + jj * h[1], lo[2] + kk * h[2]], axis=1)
    # exact box faces for boundary nodes
    xyz[ii == nx, 0] = hi[0]
    xyz[jj == ny, 1] = hi[1]
    xyz[kk == nz, 2] = hi[2]
    boundary = (ii == 0) | (ii == nx) | (jj == 0) | (jj == ny) | (kk == 0) | (kk == nz)

    ci, cj, ck = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
    ci = ci.transpose(2, 1, 0).ravel()
    cj = cj.transpose(2, 1, 0).ravel()
    ck = ck.transpose(2, 1, 0).ravel()
    tets = []
    for perm in itertools.permutations(range(3)):
        corner = np.zeros((ci.size, 3), dtype=np.int64)
        verts = [_node_id(ci, cj, ck, nx, ny)]
        for ax in perm:
            corner[:, ax] += 1
            verts.append(_node_id(ci + corner[:, 0], cj + corner[:, 1], ck + corner[:, 2], nx, ny))
        tets.append(np.stack(verts, axis=1))
    # interleave so the six tets of one cell are adjacent
    tets = np.stack(tets, axis=1).reshape(-1, 4).astype(np.int32)
    return xyz, tets, h, boundary


def jitter_interior(xyz, boundary, h, alpha, seed) -> np.ndarray:
    """Move every interior node by an independent U(-alpha*h_axis, alpha*h_axis)
    offset per coordinate (numpy default_rng(seed), one uniform draw of shape
    [n_interior, 3] in node order).  Boundary nodes stay on the box."""
    out = np.array(xyz, dtype=np.float64, copy=True)
    rng = np.random.default_rng(seed)
    idx = np.nonzero(~boundary)[0]
    u = rng.uniform(-1.0, 1.0, size=(idx.size, 3))
    out[idx] += u * (alpha * np.asarray(h, dtype=np.float64))[None, :]
    return out


def signed_volumes6(xyz, tets) -> np.ndarray:
    """Six times the signed volume of each tetrahedron (v0 origin)."""
    v = xyz[tets]
    e1 = v[:, 1] - v[:, 0]
    e2 = v[:, 2] - v[:, 0]
    e3 = v[:, 3] - v[:, 0]
    return np.einsum("ij,ij->i", e1, np.cross(e2, e3))


def orient_positive(xyz, tets) -> np.ndarray:
    """Swap the last two vertices of negatively oriented tetrahedra."""
    t = np.array(tets, copy=True)
    neg = signed_volumes6(xyz, t) < 0
    t[neg, 2], t[neg, 3] = tets[neg, 3], tets[neg, 2]
    return t


# ---------------------------------------------------------------- fields

def field_gaussian_swirl(xyz, width2=0.25):
    """omega = (-y, x, 0) * exp(-|x|^2 / width2)."""
    x, y = xyz[:, 0], xyz[:, 1]
    g = np.exp(-np.einsum("ij,ij->i", xyz, xyz) / width2)
    return np.stack([-y * g, x * g, np.zeros_like(x)], axis=1)


def field_ring(xyz, radius=1.0, sigma=0.1, gamma=1.0, z0=0.0):
    """Azimuthal vorticity of a Gaussian-core ring about the z axis:
    omega = gamma/(pi sigma^2) exp(-rho^2/sigma^2) e_theta, rho being the
    distance to the core circle (radius, in the plane z = z0)."""
    x, y, z = xyz[:, 0], xyz[:, 1], xyz[:, 2] - z0
    rc = np.hypot(x, y)
    rho2 = (rc - radius) ** 2 + z * z
    mag = gamma / (np.pi * sigma * sigma) * np.exp(-rho2 / (sigma * sigma))
    with np.errstate(invalid="ignore", divide="ignore"):
        ex = np.where(rc > 0, -y / rc, 0.0)
        ey = np.where(rc > 0, x / rc, 0.0)
    return np.stack([mag * ex, mag * ey, np.zeros_like(x)], axis=1)


def field_rings(xyz, rings, sigma):
    """Sum of Gaussian-core rings; rings = [(radius, z0, gamma), ...]."""
    out = np.zeros_like(xyz)
    for radius, z0, gamma in rings:
        out += field_ring(xyz, radius=radius, sigma=sigma, gamma=gamma, z0=z0)
    return out


def field_fourier_curl(xyz, n_modes=8, kmax=3, seed=3, normalize=True):
    """Curl of a seeded random Fourier vector potential (divergence free).

    A(x) = sum_k a_k cos(kappa_k . x + phi_k) with kappa_k = pi * n_k,
    n_k uniform in {-kmax..kmax}^3 without 0, a_k ~ N(0, I)/|kappa_k|,
    phi_k ~ U(0, 2 pi); omega = curl A analytically, scaled so that the
    largest nodal |omega| is 1."""
    rng = np.random.default_rng(seed)
    kap = []
    while len(kap) < n_modes:
        n = rng.integers(-kmax, kmax + 1, size=3)
        if np.any(n != 0):
            kap.append(np.pi * n.astype(np.float64))
    kap = np.array(kap)
    amp = rng.standard_normal((n_modes, 3)) / np.linalg.norm(kap, axis=1)[:, None]
    phase = rng.uniform(0.0, 2.0 * np.pi, size=n_modes)
    om = np.zeros_like(xyz)
    for k in range(n_modes):
        arg = xyz @ kap[k] + phase[k]
        # curl(a cos(k.x + p)) = -sin(k.x + p) k x a
        om += -np.sin(arg)[:, None] * np.cross(kap[k], amp[k])[None, :]
    if not normalize:
        return om
    scale = np.max(np.linalg.norm(om, axis=1))
    return om / scale


def field_uniform(xyz, w0):
    return np.broadcast_to(np.asarray(w0, dtype=np.float64), xyz.shape).copy()


def field_linear(xyz, w0, grad):
    """omega(x) = w0 + G x  (globally linear; exactly represented)."""
    return np.asarray(w0, dtype=np.float64)[None, :] + xyz @ np.asarray(grad, dtype=np.float64).T


# ---------------------------------------------------------------- configs

CONFIGS: Dict[str, dict] = {
    # cube [-1,1]^3, 10^3 cells, jitter 0.1 h, Gaussian swirl
    "C1": dict(lo=(-1, -1, -1), hi=(1, 1, 1), cells=(10, 10, 10), alpha=0.10, seed=1,
               field="swirl"),
    # vortex ring R=1, sigma=0.1 in a [-1.5,1.5]^2 x [-0.5,0.5] box
    "C2": dict(lo=(-1.5, -1.5, -0.5), hi=(1.5, 1.5, 0.5), cells=(64, 64, 22), alpha=0.15, seed=2,
               field="ring"),
    # precision sweep: curl of an 8-mode random Fourier potential on [-1,1]^3
    "C3": dict(lo=(-1, -1, -1), hi=(1, 1, 1), cells=(48, 48, 48), alpha=0.20, seed=3,
               field="fourier"),
    # Lagrangian run: two coaxial rings on [-1.5,1.5]^3
    "C5": dict(lo=(-1.5, -1.5, -1.5), hi=(1.5, 1.5, 1.5), cells=(80, 80, 80), alpha=0.20, seed=5,
               field="two_rings"),
}


def _field(name, xyz, seed):
    if name == "swirl":
        return field_gaussian_swirl(xyz)
    if name == "ring":
        return field_ring(xyz, radius=1.0, sigma=0.1)
    if name == "fourier":
        return field_fourier_curl(xyz, seed=seed)
    if name == "two_rings":
        return field_rings(xyz, [(1.0, -0.25, 1.0), (0.8, 0.25, 1.0)], sigma=0.08)
    raise ValueError(name)


def make_config(name: str, scale: Optional[Tuple[int, int, int]] = None, seed: Optional[int] = None) -> Mesh:
    """Build one of the named workloads.  `scale` overrides the cell counts
    (same box, same field) for reduced-size test cases."""
    c = CONFIGS[name]
    cells = tuple(scale) if scale is not None else c["cells"]
    sd = c["seed"] if seed is None else seed
    xyz, tets, h, bnd = kuhn_grid(c["lo"], c["hi"], cells)
    xyz = jitter_interior(xyz, bnd, h, c["alpha"], sd)
    tets = orient_positive(xyz, tets)
    om = _field(c["field"], xyz, sd)
    return Mesh(xyz=xyz, omega=om, tets=tets, h=h, name=name if scale is None else f"{name}@{cells}",
                boundary=bnd)


# ---------------------------------------------------------------- small inputs

def single_tet(seed=0, scale=1.0, offset=(0.0, 0.0, 0.0)):
    """One random, well-shaped tetrahedron with random nodal vorticity."""
    rng = np.random.default_rng(seed)
    base = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1]], dtype=np.float64)
    xyz = (base + 0.15 * rng.uniform(-1, 1, size=(4, 3))) * scale + np.asarray(offset)[None, :]
    tets = orient_positive(xyz, np.array([[0, 1, 2, 3]], dtype=np.int32))
    om = rng.standard_normal((4, 3))
    return Mesh(xyz=xyz, omega=om, tets=tets, h=np.array([scale] * 3), name="single_tet")


def ball_mesh(cells=12, radius=1.0, alpha=0.1, seed=7):
    """Kuhn mesh of [-r, r]^3 keeping the tetrahedra whose centroid lies in
    the ball of the given radius; nodes renumbered compactly."""
    xyz, tets, h, bnd = kuhn_grid((-radius,) * 3, (radius,) * 3, (cells,) * 3)
    xyz = jitter_interior(xyz, bnd, h, alpha, seed)
    tets = orient_positive(xyz, tets)
    cen = xyz[tets].mean(axis=1)
    keep = np.einsum("ij,ij->i", cen, cen) < radius * radius
    tets = tets[keep]
    used = np.unique(tets)
    remap = -np.ones(xyz.shape[0], dtype=np.int64)
    remap[used] = np.arange(used.size)
    return Mesh(xyz=xyz[used], omega=np.zeros((used.size, 3)), tets=remap[tets].astype(np.int32), h=h,
                name="ball")


def sphere_ball_mesh(cells=10, radius=1.0, alpha=0.1, seed=7):
    """Jittered Kuhn mesh of the cube [-1, 1]^3 carried onto the ball of the
    given radius by the smooth cube-to-sphere map
        x' = x sqrt(1 - y^2/2 - z^2/2 + y^2 z^2/3)   (and cyclically),
    which takes the cube's faces onto the sphere: every boundary node lies on
    the sphere, so the polyhedron approximates the ball to second order in h.
    Returns (xyz [n,3], tets [T,4] positively oriented, boundary [n] bool)."""
    xyz, tets, h, b = kuhn_grid((-1.0, -1.0, -1.0), (1.0, 1.0, 1.0), (cells,) * 3)
    xyz = jitter_interior(xyz, b, h, alpha, seed)
    x, y, z = xyz[:, 0], xyz[:, 1], xyz[:, 2]
    out = radius * np.stack([x * np.sqrt(1.0 - y * y / 2.0 - z * z / 2.0 + y * y * z * z / 3.0),
                             y * np.sqrt(1.0 - z * z / 2.0 - x * x / 2.0 + z * z * x * x / 3.0),
                             z * np.sqrt(1.0 - x * x / 2.0 - y * y / 2.0 + x * x * y * y / 3.0)], axis=1)
    return out, orient_positive(out, tets), b
