"""FP64 reference of the treecode far field.

Test infrastructure: only tests/, __graft_entry__.smoke() and bench.py's
cpu_baseline leg may import this package.  It shares no code with the
library.

The paper names a fast-multipole-like use of its approach as future work
(Section 4) and gives no algorithm, so what follows is this library's own
definition, written out plainly.  It replaces the all-pairs sum of the
1-point-rule pairs (the far pairs of the distance rule of Section 2 and the
Introduction) by a Barnes-Hut treecode with Cartesian multipole expansions,
the target nodes grouped in blocks of 64 that share one interaction list (a
batched treecode).  Every other pair (4-point, 11-point, ray traced) is
untouched.

Sources: the 1-point rule of every tet: point c_t = (((v0+v1)+v2)+v3)/4 and
strength W_t = |T| omega(c_t) / 4 pi (omega(c_t) the mean of the vertex
values); the pair term is W_t x (x - c_t) / |x - c_t|^3.

Tree (kd_tree): recursive median splits of a point set.  A range longer than
64 is split across the longest side of its bounding box (the first such axis
on ties) after its k smallest points by (coordinate, index), k the multiple
of 64 given by 64 * ((len // 2 + 32) // 64), at least 64 and at most len - 1.
Tet clusters are the nodes of the tree of the centroids; target blocks are
the leaves of the tree of the node positions (64 nodes each, the last one
ragged).  Every cluster and block has the sphere of its points: centre the
midpoint of their bounding box, radius the largest distance to it, both FP64.

Acceptance: with kappa = max(d_g4 hbar, largest vertex-centroid distance of
any tet) (1 + 1e-3), block B accepts cluster S iff
    |c_B - c_S|^2 >= (r_B + max(r_S / theta, r_S + kappa))^2.
Then every node x of B has |x - c_S| >= r_S / theta (the expansion converges
with ratio at most theta) and every pair of (B, S) is at distance at least
kappa, beyond the 4-point cut and not incident: the rule gives it the
1-point rule.  Traversal from the root: an accepted cluster is evaluated by
its expansion, a leaf that is not accepted pair by pair (only the pairs the
fixed rule gives the 1-point rule), anything else is opened.

Expansion of order P: with a_k(r) = (d^k (1/|r|)) / k! the Taylor
coefficients of 1/|r| and M_k = sum_t W_t (c_t - c_S)^k the cluster's
moments about its centre (multi-indices |k| <= P),
    v(x) = sum_k (-1)^|k| grad a_k(x - c_S) x M_k,
grad a_k = ((k_x + 1) a_{k+e_x}, (k_y + 1) a_{k+e_y}, (k_z + 1) a_{k+e_z}).
The coefficients follow the recurrence for the Coulomb kernel (Lindsay and
Krasny, J. Comput. Phys. 172, 2001, restated for derivatives in r):
    n |r|^2 a_k + (2n - 1) sum_i r_i a_{k-e_i} + (n - 1) sum_i a_{k-2e_i} = 0,
n = |k|, a_0 = 1/|r|.  The truncation error of one source at offset d from
the centre (|d| <= rho < R = |x - c_S|) is at most
    |W| q^(P+1) ((P+2) - (P+1) q) / (R^2 (1 - q)^2),  q = rho / R
(the degree-n Legendre term has a gradient of at most (n+1) rho^n / R^(n+2)).
"""
from __future__ import annotations

import numpy as np

LEAF = 64


# ---------------------------------------------------------------------------
# tree
def kd_tree(points, leaf=LEAF):
    """Tree of the recursive median splits of points [n, 3] (FP64).

    Returns (order, start, end, left, right): order[k] is the point at
    position k; node j covers positions [start[j], end[j]) with children
    left[j], right[j] (-1 for a leaf); node 0 is the root."""
    P = np.asarray(points, dtype=np.float64)
    n = P.shape[0]
    order = np.arange(n, dtype=np.int64)
    start, end, left, right = [0], [n], [-1], [-1]
    stack = [0]
    while stack:
        j = stack.pop()
        a, b = start[j], end[j]
        ln = b - a
        if ln <= leaf:
            continue
        idx = order[a:b]
        pts = P[idx]
        ext = pts.max(axis=0) - pts.min(axis=0)
        ax = int(np.argmax(ext))
        k = leaf * ((ln // 2 + leaf // 2) // leaf)
        k = min(max(k, leaf), ln - 1)
        s = np.lexsort((idx, pts[:, ax]))
        order[a:b] = idx[s]
        for (u, w) in ((a, a + k), (a + k, b)):
            start.append(u)
            end.append(w)
            left.append(-1)
            right.append(-1)
        left[j], right[j] = len(start) - 2, len(start) - 1
        stack += [left[j], right[j]]
    return order, np.array(start), np.array(end), np.array(left), np.array(right)


def sphere(pts):
    """Centre (midpoint of the bounding box) and radius (largest distance
    to it) of points [m, 3], FP64."""
    c = 0.5 * (pts.min(axis=0) + pts.max(axis=0))
    d = pts - c
    r2 = (d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1]) + d[:, 2] * d[:, 2]
    return c, float(np.sqrt(r2.max()))


def tet_sources(xyz, omega, tets):
    """Centroids c_t, strengths W_t and the largest vertex-centroid
    distance of the 1-point rule's sources."""
    v = xyz[tets]
    cen = (((v[:, 0] + v[:, 1]) + v[:, 2]) + v[:, 3]) * 0.25
    e = v[:, 1:] - v[:, :1]
    vol = np.abs(np.einsum("ij,ij->i", e[:, 0], np.cross(e[:, 1], e[:, 2]))) / 6.0
    w = omega[tets]
    wc = (((w[:, 0] + w[:, 1]) + w[:, 2]) + w[:, 3]) * 0.25
    W = (vol / (4.0 * np.pi))[:, None] * wc
    d = v - cen[:, None, :]
    vc2 = (d[..., 0] * d[..., 0] + d[..., 1] * d[..., 1]) + d[..., 2] * d[..., 2]
    return cen, W, float(np.sqrt(vc2.max())) if len(tets) else 0.0


def cut_distance(hbar, d_g4, vcmax):
    return max(d_g4 * hbar, vcmax) * (1.0 + 1e-3)


def accepts(cB, rB, cS, rS, theta, kappa):
    d = cB - cS
    D2 = (d[0] * d[0] + d[1] * d[1]) + d[2] * d[2]
    rho = max(rS / theta, rS + kappa)
    return D2 >= (rB + rho) * (rB + rho)


def interaction_lists(blocks, tree, csph, theta, kappa):
    """For each block (centre, radius): the clusters it accepts and the
    leaves it evaluates pair by pair."""
    _, start, end, left, right = tree
    out = []
    for (cB, rB) in blocks:
        acc, direct = [], []
        stack = [0]
        while stack:
            j = stack.pop()
            cS, rS = csph[j]
            if accepts(cB, rB, cS, rS, theta, kappa):
                acc.append(j)
            elif left[j] < 0:
                direct.append(j)
            else:
                stack += [right[j], left[j]]
        out.append((acc, direct))
    return out


# ---------------------------------------------------------------------------
# expansions
def multi_indices(order):
    """Multi-indices k = (i, j, l) with |k| <= order, by degree, then i and
    j descending."""
    return [(i, j, n - i - j) for n in range(order + 1) for i in range(n, -1, -1) for j in range(n - i, -1, -1)]


def taylor_coefficients(r, order):
    """a_k(r) = d^k (1/|r|) / k! for |k| <= order; r [m, 3].  Returns
    (a [m, count], index dict multi-index -> column)."""
    r = np.atleast_2d(np.asarray(r, dtype=np.float64))
    ks = multi_indices(order)
    col = {k: q for q, k in enumerate(ks)}
    R2 = (r[:, 0] * r[:, 0] + r[:, 1] * r[:, 1]) + r[:, 2] * r[:, 2]
    a = np.zeros((r.shape[0], len(ks)))
    a[:, 0] = 1.0 / np.sqrt(R2)
    for q in range(1, len(ks)):
        k = ks[q]
        n = sum(k)
        s = np.zeros(r.shape[0])
        for i in range(3):
            if k[i] >= 1:
                km = list(k)
                km[i] -= 1
                s += (2 * n - 1) * r[:, i] * a[:, col[tuple(km)]]
            if k[i] >= 2:
                km = list(k)
                km[i] -= 2
                s += (n - 1) * a[:, col[tuple(km)]]
        a[:, q] = -s / (n * R2)
    return a, col


def moments(cen, W, centre, order):
    """M_k = sum_t W_t (c_t - centre)^k, |k| <= order: [count, 3]."""
    d = np.asarray(cen, dtype=np.float64) - centre
    out = []
    for (i, j, l) in multi_indices(order):
        f = d[:, 0] ** i * d[:, 1] ** j * d[:, 2] ** l
        out.append(f @ W)
    return np.array(out)


def expansion_velocity(x, centre, M, order):
    """Velocity at points x [m, 3] of the order-`order` expansion of a
    cluster with moments M about centre."""
    x = np.atleast_2d(x)
    a, col = taylor_coefficients(x - centre, order + 1)
    v = np.zeros((x.shape[0], 3))
    for q, k in enumerate(multi_indices(order)):
        g = np.stack([(k[i] + 1) * a[:, col[tuple(k[c] + (c == i) for c in range(3))]] for i in range(3)], axis=1)
        v += (-1) ** sum(k) * np.cross(g, M[q])
    return v


def truncation_bound(absW_sum, rho, R, order):
    """Bound on the velocity error of the expansion of sources of total
    strength absW_sum within rho of the centre, at distance R > rho."""
    q = rho / R
    return absW_sum * q ** (order + 1) * ((order + 2) - (order + 1) * q) / (R * R * (1 - q) ** 2)


# ---------------------------------------------------------------------------
# direct 1-point-rule pairs
def g1_mask(x, cen, tets, node_ids, hbar, d_g4):
    """[m, t] True where the fixed rule gives the pair the 1-point rule: not
    incident and not (d^2 < fl32((d_g4 hbar)^2)), d^2 = ((dx dx + dy dy) +
    dz dz) in binary32 from fl32(x) - fl32(c_t), each operation rounded."""
    thr = np.float32((d_g4 * hbar) * (d_g4 * hbar))
    x32 = np.asarray(x, dtype=np.float32)
    c32 = np.asarray(cen, dtype=np.float32)
    d = x32[:, None, :] - c32[None, :, :]
    d2 = (d[..., 0] * d[..., 0] + d[..., 1] * d[..., 1]) + d[..., 2] * d[..., 2]
    inc = (tets[None, :, :] == np.asarray(node_ids)[:, None, None]).any(axis=2)
    return ~inc & ~(d2 < thr)


def direct_g1(x, node_ids, cen, W, tets, hbar, d_g4):
    """Sum of the 1-point-rule pair terms over the given tets, FP64."""
    x = np.atleast_2d(x)
    m = g1_mask(x, cen, tets, node_ids, hbar, d_g4)
    d = x[:, None, :] - cen[None, :, :]
    r2 = (d[..., 0] * d[..., 0] + d[..., 1] * d[..., 1]) + d[..., 2] * d[..., 2]
    s = np.where(m, r2 ** -1.5, 0.0)
    return (np.cross(W[None, :, :], d) * s[..., None]).sum(axis=1)


# ---------------------------------------------------------------------------
# whole far field
class Treecode:
    """Tree, clusters, blocks and cut of one mesh (FP64)."""

    def __init__(self, xyz, omega, tets, hbar, d_g4=8.0):
        self.xyz = np.asarray(xyz, dtype=np.float64)
        self.omega = np.asarray(omega, dtype=np.float64)
        self.tets = np.asarray(tets, dtype=np.int64)
        self.hbar, self.d_g4 = float(hbar), float(d_g4)
        self.cen, self.W, self.vcmax = tet_sources(self.xyz, self.omega, self.tets)
        self.kappa = cut_distance(self.hbar, self.d_g4, self.vcmax)
        self.tree = kd_tree(self.cen)
        order, start, end, _, _ = self.tree
        self.csph = [sphere(self.cen[order[start[j]:end[j]]]) for j in range(len(start))]
        norder, ns, ne, nl, _ = kd_tree(self.xyz)
        leaves = sorted((ns[j], ne[j]) for j in range(len(ns)) if nl[j] < 0)
        self.block_nodes = [norder[a:b] for (a, b) in leaves]
        self.bsph = [sphere(self.xyz[b]) for b in self.block_nodes]
        self.block_of = np.empty(len(self.xyz), dtype=np.int64)
        for q, b in enumerate(self.block_nodes):
            self.block_of[b] = q
        self._moments = {}

    def cluster_tets(self, j):
        order, start, end, _, _ = self.tree
        return order[start[j]:end[j]]

    def cluster_moments(self, j, order):
        key = (j, order)
        if key not in self._moments:
            t = self.cluster_tets(j)
            self._moments[key] = moments(self.cen[t], self.W[t], self.csph[j][0], order)
        return self._moments[key]

    def all_moments(self, order):
        """Moments [cluster, multi-index, 3] of every cluster about its
        centre: for each depth of the tree, every tet of a cluster at that
        depth adds W_t (c_t - c_S)^k to it (a bincount over the clusters)."""
        key = ("all", order)
        if key in self._moments:
            return self._moments[key]
        torder, start, end, left, right = self.tree
        nn = len(start)
        depth = np.zeros(nn, dtype=np.int64)
        for j in range(nn):
            if left[j] >= 0:
                depth[left[j]] = depth[right[j]] = depth[j] + 1
        ks = multi_indices(order)
        ctr = np.array([c for (c, _) in self.csph])
        M = np.zeros((nn, len(ks), 3))
        for dlev in range(depth.max() + 1):
            ids = np.nonzero(depth == dlev)[0]
            lens = end[ids] - start[ids]
            anc = np.repeat(ids, lens)
            pos = np.concatenate([np.arange(start[j], end[j]) for j in ids])
            t = torder[pos]
            d = self.cen[t] - ctr[anc]
            for q, (i, j2, l) in enumerate(ks):
                f = d[:, 0] ** i * d[:, 1] ** j2 * d[:, 2] ** l
                for c in range(3):
                    M[:, q, c] += np.bincount(anc, weights=f * self.W[t, c], minlength=nn)
        self._moments[key] = M
        return M

    def lists(self, theta, blocks):
        return interaction_lists([self.bsph[b] for b in blocks], self.tree, self.csph, theta, self.kappa)

    def far(self, theta, order, targets):
        """Treecode far field (the 1-point-rule pairs) at node indices
        targets, FP64 [m, 3]: every (target, accepted cluster) expansion in
        one batch, then the direct leaves block by block."""
        targets = np.asarray(targets, dtype=np.int64)
        out = np.zeros((len(targets), 3))
        blocks = np.unique(self.block_of[targets])
        lists = self.lists(theta, blocks)
        M = self.all_moments(order)
        ctr = np.array([c for (c, _) in self.csph])
        rows, clus = [], []
        for b, (acc, direct) in zip(blocks, lists):
            r = np.nonzero(self.block_of[targets] == b)[0]
            if acc:
                rows.append(np.repeat(r, len(acc)))
                clus.append(np.tile(np.asarray(acc, dtype=np.int64), len(r)))
            if direct:
                ids = targets[r]
                t = np.concatenate([self.cluster_tets(j) for j in direct])
                out[r] += direct_g1(self.xyz[ids], ids, self.cen[t], self.W[t], self.tets[t], self.hbar, self.d_g4)
        if rows:
            rows = np.concatenate(rows)
            clus = np.concatenate(clus)
            for q in range(0, len(rows), 1 << 16):
                rr, cc = rows[q:q + (1 << 16)], clus[q:q + (1 << 16)]
                a, col = taylor_coefficients(self.xyz[targets[rr]] - ctr[cc], order + 1)
                v = np.zeros((len(rr), 3))
                for qk, k in enumerate(multi_indices(order)):
                    g = np.stack([(k[i] + 1) * a[:, col[tuple(k[c] + (c == i) for c in range(3))]]
                                  for i in range(3)], axis=1)
                    v += (-1) ** sum(k) * np.cross(g, M[cc, qk])
                np.add.at(out, rr, v)
        return out

    def direct_far(self, targets):
        """The all-pairs sum the treecode replaces, FP64 [m, 3]."""
        targets = np.asarray(targets, dtype=np.int64)
        out = np.zeros((len(targets), 3))
        step = max(1, (1 << 23) // max(1, len(self.tets)))
        for q in range(0, len(targets), step):
            ids = targets[q:q + step]
            out[q:q + step] = direct_g1(self.xyz[ids], ids, self.cen, self.W, self.tets, self.hbar, self.d_g4)
        return out
