"""FP64 pair features of the rule selector (test infrastructure only),
written from their definition:
  d = |c| with c = centroid - x; h_T, h_min longest / shortest edge;
  lambda_j barycentric coordinates of x; n_f outward unit face normals;
  6V the absolute volume triple product.
  [d/h_T, d/hbar, h_T/h_min, hbar/d, sort_desc(lambda h_T/d) (4),
   sort_desc(n_f . (-c/d)) (4), incident, 6V/h_T^3, min_f dist(x, plane_f)/h_T, 1]
"""
import numpy as np


def pair_features(x, tv, hbar, incident=False):
    x = np.asarray(x, dtype=np.float64)
    v = np.asarray(tv, dtype=np.float64)
    c = v.mean(axis=0) - x
    d = np.linalg.norm(c)
    edges = [np.linalg.norm(v[j] - v[i]) for i in range(4) for j in range(i + 1, 4)]
    hT, hmin = max(edges), min(edges)
    # barycentric coordinates of x: solve sum lambda_j v_j = x, sum lambda_j = 1
    A = np.vstack([v.T, np.ones(4)])
    lam = np.linalg.solve(A, np.append(x, 1.0))
    six_v = abs(np.linalg.det(np.stack([v[1] - v[0], v[2] - v[0], v[3] - v[0]])))
    cos, dist = [], []
    for f in range(4):
        p, q, r = [j for j in range(4) if j != f]
        n = np.cross(v[q] - v[p], v[r] - v[p])
        n /= np.linalg.norm(n)
        if np.dot(n, v[f] - v[p]) > 0:
            n = -n
        cos.append(np.dot(n, -c / d))
        dist.append(abs(np.dot(n, x - v[p])))
    return np.concatenate([[d / hT, d / hbar, hT / hmin, hbar / d], np.sort(lam * hT / d)[::-1],
                           np.sort(cos)[::-1], [1.0 if incident else 0.0, six_v / hT ** 3, min(dist) / hT, 1.0]])


def pair_features_batch(X, TV, hbar, incident):
    """pair_features for P pairs at once (X [P,3], TV [P,4,3], incident [P]),
    the same definition written with array operations; checked against
    pair_features pair by pair in the tests."""
    X = np.asarray(X, dtype=np.float64)
    V = np.asarray(TV, dtype=np.float64)
    P = X.shape[0]
    c = V.mean(axis=1) - X
    d = np.linalg.norm(c, axis=1)
    edges = np.stack([np.linalg.norm(V[:, j] - V[:, i], axis=1) for i in range(4) for j in range(i + 1, 4)], axis=1)
    hT, hmin = edges.max(axis=1), edges.min(axis=1)
    A = np.concatenate([V.transpose(0, 2, 1), np.ones((P, 1, 4))], axis=1)
    rhs = np.concatenate([X, np.ones((P, 1))], axis=1)
    lam = np.linalg.solve(A, rhs[:, :, None])[:, :, 0]
    six_v = np.abs(np.linalg.det(np.stack([V[:, 1] - V[:, 0], V[:, 2] - V[:, 0], V[:, 3] - V[:, 0]], axis=1)))
    cos = np.empty((P, 4))
    dist = np.empty((P, 4))
    u = -c / d[:, None]
    for f in range(4):
        p, q, r = [j for j in range(4) if j != f]
        n = np.cross(V[:, q] - V[:, p], V[:, r] - V[:, p])
        n /= np.linalg.norm(n, axis=1)[:, None]
        flip = np.einsum("ij,ij->i", n, V[:, f] - V[:, p]) > 0
        n[flip] = -n[flip]
        cos[:, f] = np.einsum("ij,ij->i", n, u)
        dist[:, f] = np.abs(np.einsum("ij,ij->i", n, X - V[:, p]))
    lam_s = -np.sort(-(lam * (hT / d)[:, None]), axis=1)
    cos_s = -np.sort(-cos, axis=1)
    inc = np.asarray(incident, dtype=np.float64).reshape(P)
    return np.concatenate([np.stack([d / hT, d / hbar, hT / hmin, hbar / d], axis=1), lam_s, cos_s,
                           np.stack([inc, six_v / hT ** 3, dist.min(axis=1) / hT, np.ones(P)], axis=1)], axis=1)
