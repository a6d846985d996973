"""FP64 kinematics of the Lagrangian application (test infrastructure only).

The paper's method evaluates the velocity; its application (Sections 1
and 3) moves the vorticity-carrying nodes with it and, in a vortex method,
stretches their vorticity, (w . grad) v.  The paper gives no discretisation
of the stretching term.  This module follows the library's stated one,
written from its definition:

  * on a tetrahedron the piecewise-linear interpolant of nodal velocities
    has a constant gradient G with G (x_j - x_0) = v_j - v_0 for j = 1..3;
  * at a node, the gradients of its tetrahedra averaged with their volumes
    as weights (zero at a node of no tetrahedron);
  * the stretching rate of node i is G_i w_i;
  * Heun (RK2) on the node positions, and with stretching on the vorticity:
    k1 = f(y); y* = y + dt k1; k2 = f(y*); y <- y + dt/2 (k1 + k2).
"""
import numpy as np


def tet_gradients(xyz, tets, vel):
    """Per tetrahedron: the interpolant's gradient G [T,3,3] (G[t,a,b] =
    dv_a/dx_b) and the volume [T]."""
    X = np.asarray(xyz, dtype=np.float64)[np.asarray(tets)]
    V = np.asarray(vel, dtype=np.float64)[np.asarray(tets)]
    E = X[:, 1:, :] - X[:, :1, :]  # rows: edge vectors e_j = x_j - x_0
    D = V[:, 1:, :] - V[:, :1, :]  # rows: v_j - v_0
    # G e_j = d_j for each j  <=>  E G^T = D (rows of E are the e_j)
    Gt = np.linalg.solve(E, D)
    vol = np.abs(np.linalg.det(E)) / 6.0
    return np.transpose(Gt, (0, 2, 1)), vol


def nodal_velocity_gradient(xyz, tets, vel):
    """Volume-weighted mean of the tetrahedra's gradients at every node [n,3,3]."""
    n = np.asarray(xyz).shape[0]
    G, vol = tet_gradients(xyz, tets, vel)
    num = np.zeros((n, 3, 3))
    den = np.zeros(n)
    for j in range(4):
        np.add.at(num, np.asarray(tets)[:, j], G * vol[:, None, None])
        np.add.at(den, np.asarray(tets)[:, j], vol)
    out = np.zeros_like(num)
    has = den > 0
    out[has] = num[has] / den[has, None, None]
    return out


def stretching(grad, omega):
    """(w . grad) v at every node: G_i w_i."""
    return np.einsum("iab,ib->ia", grad, np.asarray(omega, dtype=np.float64))


def heun(y, f, dt):
    """One Heun step of dy/dt = f(y) for a tuple of arrays y."""
    k1 = f(y)
    ys = tuple(a + dt * k for a, k in zip(y, k1))
    k2 = f(ys)
    return tuple(a + 0.5 * dt * (p + q) for a, p, q in zip(y, k1, k2))


def lagrangian_step(xyz, omega, tets, dt, velocity, stretch=True):
    """One Heun step of the nodes (and, with stretch, their vorticity);
    velocity(xyz, omega) returns the nodal velocities [n,3]."""
    def f(y):
        x, w = y
        v = velocity(x, w)
        s = stretching(nodal_velocity_gradient(x, tets, v), w) if stretch else np.zeros_like(w)
        return v, s

    return heun((np.asarray(xyz, dtype=np.float64), np.asarray(omega, dtype=np.float64)), f, dt)
