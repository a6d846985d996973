"""Pins of the treecode far field's FP64 reference (oracle/treecode.py).

Each check is against something other than the reference itself: the
Taylor coefficients against the power series of (R^2 + 2 r.h + h.h)^(-1/2)
built by polynomial products and against Laplace's equation; expansions
against the direct sum within the Legendre truncation bound; the 1-point
mask against the C oracle's own rule decisions; the acceptance test against
those decisions on every accepted pair; the tree against its definition by
brute force.
"""
import itertools
import math

import numpy as np
import pytest

import oracle
import workloads as W
from oracle import treecode as TC


def _poly_mul(a, b, D):
    out = np.zeros_like(a)
    nz = [(i, j, l) for i in range(D + 1) for j in range(D + 1 - i) for l in range(D + 1 - i - j)]
    for (i, j, l) in nz:
        if a[i, j, l] == 0.0:
            continue
        for (p, q, s) in nz:
            if i + p + j + q + l + s <= D and b[p, q, s] != 0.0:
                out[i + p, j + q, l + s] += a[i, j, l] * b[p, q, s]
    return out


def _series_of_inverse_distance(r, D):
    """Coefficients c[i, j, l] of h^(i,j,l) in 1/|r + h| up to degree D."""
    R2 = float(r @ r)
    u = np.zeros((D + 1,) * 3)
    for c in range(3):
        e = [0, 0, 0]
        e[c] = 1
        u[tuple(e)] = 2.0 * r[c] / R2
        e[c] = 2
        u[tuple(e)] = 1.0 / R2
    out = np.zeros_like(u)
    term = np.zeros_like(u)
    term[0, 0, 0] = 1.0
    for j in range(D + 1):
        binom = math.prod(-0.5 - q for q in range(j)) / math.factorial(j)
        out += binom * term
        term = _poly_mul(term, u, D)
    return out / math.sqrt(R2)


def test_taylor_coefficients_match_the_power_series():
    rng = np.random.default_rng(11)
    D = 7
    for _ in range(4):
        r = rng.normal(size=3)
        a, col = TC.taylor_coefficients(r, D)
        c = _series_of_inverse_distance(r, D)
        for k in TC.multi_indices(D):
            assert abs(a[0, col[k]] - c[k]) <= 1e-12 * max(1.0, abs(c[k])), k


def test_taylor_coefficients_are_harmonic():
    rng = np.random.default_rng(12)
    r = rng.normal(size=(5, 3))
    D = 8
    a, col = TC.taylor_coefficients(r, D)
    scale = np.abs(a).max(axis=1)
    for k in TC.multi_indices(D - 2):
        lap = sum((k[c] + 1) * (k[c] + 2) * a[:, col[tuple(k[i] + 2 * (i == c) for i in range(3))]] for c in range(3))
        assert np.all(np.abs(lap) <= 1e-11 * scale), k


def test_expansion_error_within_the_truncation_bound():
    rng = np.random.default_rng(13)
    centre = np.array([0.1, -0.2, 0.3])
    d = rng.uniform(-1, 1, size=(60, 3))
    d *= 0.3 / np.linalg.norm(d, axis=1).max()
    src = centre + d
    Wt = rng.normal(size=(60, 3))
    rho = np.linalg.norm(d, axis=1).max()
    absW = np.linalg.norm(Wt, axis=1).sum()
    dirs = rng.normal(size=(12, 3))
    dirs /= np.linalg.norm(dirs, axis=1)[:, None]
    for R in (0.5, 0.8, 1.5, 3.0):
        x = centre + R * dirs
        dd = x[:, None, :] - src[None]
        exact = (np.cross(Wt[None], dd) * (np.linalg.norm(dd, axis=2) ** -3)[..., None]).sum(axis=1)
        prev = None
        for P in range(0, 9):
            M = TC.moments(src, Wt, centre, P)
            err = np.linalg.norm(TC.expansion_velocity(x, centre, M, P) - exact, axis=1).max()
            bound = TC.truncation_bound(absW, rho, R, P)
            assert err <= bound * (1 + 1e-9) + 1e-13, (R, P, err, bound)
            if prev is not None and R >= 1.5:
                assert err < prev, (R, P)
            prev = err
    # a dropped term of any order shows: order 8 at q = 0.1 is within 1e-8
    # of the exact value relative to its size
    x = centre + 3.0 * dirs
    M = TC.moments(src, Wt, centre, 8)
    dd = x[:, None, :] - src[None]
    exact = (np.cross(Wt[None], dd) * (np.linalg.norm(dd, axis=2) ** -3)[..., None]).sum(axis=1)
    assert np.abs(TC.expansion_velocity(x, centre, M, 8) - exact).max() < 1e-8 * np.abs(exact).max()


def test_kd_tree_is_the_median_split_of_its_definition():
    rng = np.random.default_rng(14)
    pts = np.round(rng.uniform(-1, 1, size=(1000, 3)) * 8) / 8  # many equal coordinates
    pts[:, 2] *= 3.0
    order, start, end, left, right = TC.kd_tree(pts)
    leaves = [j for j in range(len(start)) if left[j] < 0]
    cover = np.concatenate([order[start[j]:end[j]] for j in sorted(leaves, key=lambda j: start[j])])
    assert np.array_equal(np.sort(cover), np.arange(len(pts)))
    assert all(end[j] - start[j] <= 64 for j in leaves)
    for j in range(len(start)):
        if left[j] < 0:
            assert end[j] - start[j] <= 64
            continue
        a, b = start[j], end[j]
        ln = b - a
        k = min(max(64 * ((ln // 2 + 32) // 64), 64), ln - 1)
        assert (start[left[j]], end[left[j]], start[right[j]], end[right[j]]) == (a, a + k, a + k, b)
        sub = pts[order[a:b]]
        ext = sub.max(axis=0) - sub.min(axis=0)
        ax = [c for c in range(3) if ext[c] == ext.max()][0]
        lo = [(pts[i, ax], i) for i in order[a:a + k]]
        hi = [(pts[i, ax], i) for i in order[a + k:b]]
        assert max(lo) < min(hi)


def _c1_with_small_cuts():
    m = W.make_config("C1")
    pol = oracle.make_policy("fixed", near_cut=1.0, d_g11=1.5, d_g4=2.0)
    hbar = oracle.mean_edge(m.xyz, m.tets)
    return m, pol, hbar


def test_one_point_mask_is_the_rule_of_the_oracle():
    m, pol, hbar = _c1_with_small_cuts()
    _, rules = oracle.evaluate(m.xyz, m.omega, m.tets, pol, return_rules=True)
    cen, _, _ = TC.tet_sources(m.xyz, m.omega, m.tets)
    ids = np.arange(len(m.xyz))
    mask = np.concatenate([TC.g1_mask(m.xyz[q:q + 200], cen, m.tets, ids[q:q + 200], hbar, 2.0)
                           for q in range(0, len(ids), 200)])
    assert np.array_equal(mask, rules == oracle.RULE_G1)
    assert mask.sum() > 0 and (~mask).sum() > 0


def test_accepted_pairs_are_one_point_rule_pairs():
    m, pol, hbar = _c1_with_small_cuts()
    _, rules = oracle.evaluate(m.xyz, m.omega, m.tets, pol, return_rules=True)
    tc = TC.Treecode(m.xyz, m.omega, m.tets, hbar, d_g4=2.0)
    blocks = list(range(len(tc.block_nodes)))
    n_acc = 0
    for b, (acc, direct) in zip(blocks, tc.lists(0.7, blocks)):
        nodes = tc.block_nodes[b]
        for j in acc:
            t = tc.cluster_tets(j)
            assert np.all(rules[np.ix_(nodes, t)] == oracle.RULE_G1), (b, j)
            n_acc += len(t) * len(nodes)
        # the accepted clusters and direct leaves cover every tet once
        cover = np.concatenate([tc.cluster_tets(j) for j in acc + direct])
        assert np.array_equal(np.sort(cover), np.arange(len(m.tets)))
    assert n_acc > 0.2 * len(m.xyz) * len(m.tets)


def test_treecode_converges_to_the_direct_sum_within_the_bound():
    m, pol, hbar = _c1_with_small_cuts()
    tc = TC.Treecode(m.xyz, m.omega, m.tets, hbar, d_g4=2.0)
    rng = np.random.default_rng(15)
    targets = rng.choice(len(m.xyz), 96, replace=False)
    exact = tc.direct_far(targets)
    scale = np.abs(exact).max()
    errs = []
    for P in (1, 2, 4, 6, 8):
        far = tc.far(0.5, P, targets)
        e = np.linalg.norm(far - exact, axis=1)
        # per node: within the sum of the accepted clusters' bounds
        for q, i in enumerate(targets):
            b = tc.block_of[i]
            acc, _ = tc.lists(0.5, [b])[0]
            bound = 0.0
            for j in acc:
                t = tc.cluster_tets(j)
                cS, _ = tc.csph[j]
                rho = np.linalg.norm(tc.cen[t] - cS, axis=1).max()
                R = np.linalg.norm(m.xyz[i] - cS)
                bound += TC.truncation_bound(np.linalg.norm(tc.W[t], axis=1).sum(), rho, R, P)
            assert e[q] <= bound * (1 + 1e-9) + 1e-14 * scale, (P, i)
        errs.append(e.max() / scale)
    assert all(b < a for a, b in zip(errs, errs[1:])), errs
    assert errs[-1] < 1e-6, errs


def test_vanishing_theta_is_the_direct_sum():
    m, pol, hbar = _c1_with_small_cuts()
    tc = TC.Treecode(m.xyz, m.omega, m.tets, hbar, d_g4=2.0)
    targets = np.arange(0, len(m.xyz), 7)
    far = tc.far(1e-9, 4, targets)
    exact = tc.direct_far(targets)
    assert np.abs(far - exact).max() <= 1e-13 * np.abs(exact).max()


def test_direct_sum_is_the_oracles_one_point_share():
    """The direct 1-point sum equals the C oracle's own 1-point pair terms
    summed over the pairs its rule gives the 1-point rule."""
    m, pol, hbar = _c1_with_small_cuts()
    targets = np.array([5, 400, 777])
    _, rules = oracle.evaluate(m.xyz, m.omega, m.tets, pol, targets=targets, return_rules=True)
    tc = TC.Treecode(m.xyz, m.omega, m.tets, hbar, d_g4=2.0)
    got = tc.direct_far(targets)
    for q, i in enumerate(targets):
        ref = np.zeros(3)
        for t in np.nonzero(rules[q] == oracle.RULE_G1)[0]:
            ids = m.tets[t]
            ref += oracle.pair(m.xyz[i], m.xyz[ids], m.omega[ids], oracle.RULE_G1)
        assert np.abs(got[q] - ref).max() <= 1e-13 * np.abs(ref).max()
