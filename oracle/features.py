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
