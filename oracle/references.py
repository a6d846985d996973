"""Exact references that pin the oracle (test infrastructure only).

Nothing here runs the ray-tracing or Gauss-rule code of ``bs_oracle.c``;
each function computes the quantity another way:

* simplex_moment: closed-form integral of a barycentric monomial over a
  tetrahedron (pins the tetrahedral Gauss rules).
* ball_line_sum / cube_line_sum: the angular quadrature of eq. 3 applied to
  the exact line integrals through an analytic ball or box (uniform or
  globally linear vorticity).  On any tetrahedral mesh of the box, the sum
  over tetrahedra of the per-tetrahedron chords reproduces these line
  integrals up to rounding, whatever the mesh.
* ball_uniform_velocity / box_uniform_velocity: closed forms of the
  Biot-Savart integral of uniform vorticity in a ball (omega x x / 3 inside)
  and in a box (surface form with the rectangle potential).
* tet_cone_brute_force: the exact velocity of one tetrahedron with linear
  vorticity by the signed cone decomposition from the target point (radial
  integral exact, face integrals by a high-order collapsed Gauss rule).
* tet_subdivision: the volume integral by recursive 8-way subdivision with a
  degree-4 rule per sub-tetrahedron (for targets away from the element).
* gaussian_vortex: a smooth, compactly decaying vorticity with an analytic
  velocity (for the convergence-under-refinement test).
* hill_vorticity / hill_velocity: Hill's spherical vortex (Section 3.1), the
  paper's test problem, with its closed-form velocity.
"""
from __future__ import annotations

import math
from typing import Tuple

import numpy as np

FOUR_PI = 4.0 * math.pi


# ---------------------------------------------------------------- simplex

def simplex_moment(e) -> float:
    """Mean over a tetrahedron of prod_j lambda_j^e_j:
    3! prod e_j! / (sum e_j + 3)!."""
    e = [int(v) for v in e]
    num = 6.0
    for v in e:
        num *= math.factorial(v)
    return num / math.factorial(sum(e) + 3)


# ---------------------------------------------------------------- line sums

def ball_line_sum(s, k, x, w0, a=1.0):
    """sum_l k_l * integral over the line x + R s_l of sgn(R) s_l x w0, for
    uniform w0 inside the ball |y| < a (x inside the ball)."""
    x = np.asarray(x, dtype=np.float64)
    xs = s @ x
    disc = xs * xs - (x @ x) + a * a
    rp = -xs + np.sqrt(disc)
    rm = -xs - np.sqrt(disc)
    # integral of sgn(R) over [rm, rp] with rm < 0 < rp is rp + rm
    L = rp + rm
    return np.sum((k * L)[:, None] * np.cross(s, np.asarray(w0)[None, :]), axis=0)


def _box_exit(x, d, lo, hi):
    """Distance from x (inside the closed box) to the boundary along +d."""
    t = np.full(d.shape[0], np.inf)
    for c in range(3):
        dc = d[:, c]
        with np.errstate(divide="ignore", invalid="ignore"):
            tp = np.where(dc > 0, (hi[c] - x[c]) / dc, np.inf)
            tm = np.where(dc < 0, (lo[c] - x[c]) / dc, np.inf)
        t = np.minimum(t, np.minimum(tp, tm))
    return np.maximum(t, 0.0)


def cube_line_sum(s, k, x, lo, hi, w0, grad=None):
    """sum_l k_l * integral over the line x + R s_l inside the box [lo, hi]
    of sgn(R) s_l x omega(x + R s_l), omega(y) = w0 + G y (G = grad)."""
    x = np.asarray(x, dtype=np.float64)
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    G = np.zeros((3, 3)) if grad is None else np.asarray(grad, dtype=np.float64)
    rp = _box_exit(x, s, lo, hi)
    rm = _box_exit(x, -s, lo, hi)
    wx = np.asarray(w0, dtype=np.float64) + G @ x
    # integral of sgn(R) (w(x) + R G s) over [-rm, rp]
    vec = (rp - rm)[:, None] * wx[None, :] + (0.5 * (rp * rp + rm * rm))[:, None] * (s @ G.T)
    return np.sum(k[:, None] * np.cross(s, vec), axis=0)


# ---------------------------------------------------------------- closed forms

def ball_uniform_velocity(x, w0):
    """Uniform vorticity w0 in a ball, x inside: v = w0 x x / 3."""
    return np.cross(np.asarray(w0, dtype=np.float64), np.asarray(x, dtype=np.float64)) / 3.0


def _rect_inv_r(X, u1, u2, v1, v2):
    """Integral over the rectangle [u1,u2]x[v1,v2] of 1/sqrt(X^2+u^2+v^2)."""

    def F(u, v):
        R = math.sqrt(X * X + u * u + v * v)
        val = 0.0
        if u != 0.0:
            val += u * math.log(v + R) if v + R > 0 else 0.0
        if v != 0.0:
            val += v * math.log(u + R) if u + R > 0 else 0.0
        if X != 0.0 and R > 0.0:
            val -= X * math.atan(u * v / (X * R))
        return val

    return F(u2, v2) - F(u1, v2) - F(u2, v1) + F(u1, v1)


def box_surface_g(x, lo, hi):
    """g(x) = closed-surface integral of n_hat / |x - y| over the box."""
    x = np.asarray(x, dtype=np.float64)
    g = np.zeros(3)
    for c in range(3):
        a, b = [d for d in range(3) if d != c]
        u1, u2 = lo[a] - x[a], hi[a] - x[a]
        v1, v2 = lo[b] - x[b], hi[b] - x[b]
        g[c] += _rect_inv_r(hi[c] - x[c], u1, u2, v1, v2)  # outward +e_c
        g[c] -= _rect_inv_r(lo[c] - x[c], u1, u2, v1, v2)  # outward -e_c
    return g


def box_uniform_velocity(x, lo, hi, w0):
    """Biot-Savart velocity of uniform w0 filling the box [lo, hi]:
    v = -(1/4pi) (integral of (x - y)/|x - y|^3 dV) x w0 and
    integral (x - y)/|x-y|^3 dV = -grad_x integral 1/|x-y| dV = surface
    integral of n_hat/|x - y| dS (outward normal)."""
    g = box_surface_g(x, lo, hi)
    return -np.cross(g, np.asarray(w0, dtype=np.float64)) / FOUR_PI


# ---------------------------------------------------------------- brute force

def _tri_rule(order):
    """Collapsed (Duffy) Gauss rule on the reference triangle
    {(u, v): u, v >= 0, u + v <= 1}: points (u, v) and weights (sum 1/2)."""
    t, w = np.polynomial.legendre.leggauss(order)
    t = 0.5 * (t + 1.0)
    w = 0.5 * w
    a, b = np.meshgrid(t, t, indexing="ij")
    wa, wb = np.meshgrid(w, w, indexing="ij")
    u = a * (1.0 - b)
    v = a * b
    ww = wa * wb * a
    return np.stack([u.ravel(), v.ravel()], axis=1), ww.ravel()


def tet_cone_brute_force(x, tv, tw, order=48):
    """Velocity at x of one tetrahedron (vertices tv [4,3], linear vorticity
    with vertex values tw [4,3]).

    The tetrahedron is the signed sum of the four cones from x over its faces
    (sign +1 when x lies on the inner side of the face plane).  Over a cone
    the radial integral of the linear vorticity is exact, leaving
    (1/4pi) int_F (p - x) x (omega(x) + omega(p))/2 * h_F / |p - x|^3 dA_p,
    h_F the distance from x to the face plane; faces through x contribute
    nothing."""
    x = np.asarray(x, dtype=np.float64)
    tv = np.asarray(tv, dtype=np.float64)
    tw = np.asarray(tw, dtype=np.float64)
    # linear vorticity extended to all space: omega(y) = sum lambda_j(y) w_j
    A = np.vstack([tv.T, np.ones(4)])
    lam_x = np.linalg.solve(A, np.append(x, 1.0))
    om_x = lam_x @ tw
    pts, wts = _tri_rule(order)
    out = np.zeros(3)
    cen = tv.mean(axis=0)
    for f in range(4):
        idx = [j for j in range(4) if j != f]
        a, b, c = tv[idx]
        n = np.cross(b - a, c - a)
        area2 = np.linalg.norm(n)
        nh = n / area2
        dist = float(np.dot(x - a, nh))
        if dist == 0.0:
            continue
        # inner side of the face plane is where the opposite vertex lies
        sign = 1.0 if np.sign(dist) == np.sign(np.dot(cen - a, nh)) else -1.0
        p = a[None, :] + pts[:, 0:1] * (b - a)[None, :] + pts[:, 1:2] * (c - a)[None, :]
        lam_p = np.zeros((p.shape[0], 4))
        lam_p[:, idx[0]] = 1.0 - pts[:, 0] - pts[:, 1]
        lam_p[:, idx[1]] = pts[:, 0]
        lam_p[:, idx[2]] = pts[:, 1]
        om_p = lam_p @ tw
        d = p - x[None, :]
        r3 = np.linalg.norm(d, axis=1) ** 3
        integ = np.cross(d, 0.5 * (om_x[None, :] + om_p)) * (abs(dist) / r3)[:, None]
        out += sign * (wts * area2) @ integ
    return out / FOUR_PI


def _keast11():
    c = (1.0 + math.sqrt(5.0 / 14.0)) / 4.0
    d = (1.0 - math.sqrt(5.0 / 14.0)) / 4.0
    lam = [[0.25] * 4]
    w = [-148.0 / 1875.0]
    for v in range(4):
        lam.append([11.0 / 14.0 if j == v else 1.0 / 14.0 for j in range(4)])
        w.append(343.0 / 7500.0)
    for i in range(4):
        for j in range(i + 1, 4):
            lam.append([c if l in (i, j) else d for l in range(4)])
            w.append(56.0 / 375.0)
    return np.array(lam), np.array(w)


def _bey_children(t):
    """8 children of tetrahedra t [m,4,3] by Bey's red refinement."""
    x0, x1, x2, x3 = t[:, 0], t[:, 1], t[:, 2], t[:, 3]
    x01, x02, x03 = (x0 + x1) / 2, (x0 + x2) / 2, (x0 + x3) / 2
    x12, x13, x23 = (x1 + x2) / 2, (x1 + x3) / 2, (x2 + x3) / 2
    kids = [
        (x0, x01, x02, x03), (x01, x1, x12, x13), (x02, x12, x2, x23), (x03, x13, x23, x3),
        (x01, x02, x03, x13), (x01, x02, x12, x13), (x02, x03, x13, x23), (x02, x12, x13, x23),
    ]
    return np.concatenate([np.stack(k, axis=1) for k in kids], axis=0)


def tet_subdivision(x, tv, tw, levels=4):
    """Volume integral of one tetrahedron by `levels` rounds of 8-way
    subdivision and the degree-4 (11-point) rule on every sub-tetrahedron.
    For targets away from the element (the integrand is then smooth)."""
    x = np.asarray(x, dtype=np.float64)
    tv = np.asarray(tv, dtype=np.float64)
    tw = np.asarray(tw, dtype=np.float64)
    A = np.vstack([tv.T, np.ones(4)])
    Ainv = np.linalg.inv(A)
    lam, w = _keast11()
    t = tv[None, :, :]
    for _ in range(levels):
        t = _bey_children(t)
    pts = np.einsum("qj,mjc->mqc", lam, t)  # [m, q, 3]
    e1 = t[:, 1] - t[:, 0]
    vol = np.abs(np.einsum("ij,ij->i", e1, np.cross(t[:, 2] - t[:, 0], t[:, 3] - t[:, 0]))) / 6.0
    bary = np.einsum("ij,mqj->mqi", Ainv, np.concatenate([pts, np.ones(pts.shape[:2] + (1,))], axis=2))
    om = bary @ tw
    r = x[None, None, :] - pts
    r3 = np.linalg.norm(r, axis=2) ** 3
    integ = -np.cross(r, om) / r3[..., None] / FOUR_PI
    return np.einsum("m,q,mqc->c", vol, w, integ)


# ---------------------------------------------------------------- Hill's vortex

def hill_vorticity(xyz, A=1.0, a=1.0):
    """Hill's spherical vortex (Section 3.1): azimuthal vorticity
    omega_theta = A r (r the distance from the z axis) inside the sphere of
    radius a, i.e. omega = A (-y, x, 0) there, zero outside."""
    xyz = np.asarray(xyz, dtype=np.float64)
    inside = np.einsum("ij,ij->i", xyz, xyz) < a * a
    om = A * np.stack([-xyz[:, 1], xyz[:, 0], np.zeros(len(xyz))], axis=1)
    return np.where(inside[:, None], om, 0.0)


def hill_velocity(xyz, A=1.0, a=1.0):
    """Velocity of Hill's vortex in the frame where the fluid is at rest far
    away (the form of Section 3.1's closed form with its misprints corrected):
    inside (|x| < a), in cylindrical (r, z) components,
        u_r = A r z / 5,   u_z = (A / 5) (5 a^2 / 3 - 2 r^2 - z^2);
    outside, the potential flow of a sphere of radius a moving along +z at
    U = 2 A a^2 / 15: u = U a^3 / (2 R^3) (3 (e.x) x / R^2 - e) with
    e = (0, 0, 1), R = |x|.  (Its curl inside is A r e_theta, it is
    divergence free, and both normal and tangential components match across
    R = a.)"""
    xyz = np.asarray(xyz, dtype=np.float64)
    x, y, z = xyz[:, 0], xyz[:, 1], xyz[:, 2]
    R2 = x * x + y * y + z * z
    inside = R2 < a * a
    u_in = np.stack([A * x * z / 5.0, A * y * z / 5.0, A / 5.0 * (5.0 * a * a / 3.0 - 2.0 * (x * x + y * y) - z * z)],
                    axis=1)
    U = 2.0 * A * a * a / 15.0
    with np.errstate(invalid="ignore", divide="ignore"):
        R = np.sqrt(R2)
        f = U * a ** 3 / (2.0 * R ** 3)
        u_out = np.stack([f * 3.0 * z * x / R2, f * 3.0 * z * y / R2, f * (3.0 * z * z / R2 - 1.0)], axis=1)
    return np.where(inside[:, None], u_in, u_out)


# ---------------------------------------------------------------- smooth field

def gaussian_vortex(xyz, sigma=0.3):
    """psi = (0, 0, f), f = exp(-|x|^2 / sigma^2): velocity v = curl psi and
    vorticity omega = curl v (divergence free, Gaussian decay), both
    analytic.  Returns (omega, v)."""
    x, y, z = xyz[:, 0], xyz[:, 1], xyz[:, 2]
    s2 = sigma * sigma
    f = np.exp(-(x * x + y * y + z * z) / s2)
    fx, fy = -2 * x / s2 * f, -2 * y / s2 * f
    v = np.stack([fy, -fx, np.zeros_like(x)], axis=1)
    # omega = (d_x d_z f, d_y d_z f, -(d_xx + d_yy) f)
    fxz = 4 * x * z / (s2 * s2) * f
    fyz = 4 * y * z / (s2 * s2) * f
    fxx = (4 * x * x / (s2 * s2) - 2 / s2) * f
    fyy = (4 * y * y / (s2 * s2) - 2 / s2) * f
    om = np.stack([fxz, fyz, -(fxx + fyy)], axis=1)
    return om, v
