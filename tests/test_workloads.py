"""Input generators: counts, orientation and conformity of the Kuhn meshes."""
import numpy as np
import pytest

import workloads as W

COUNTS = {"C1": (1331, 6000), "C2": (97175, 540672), "C3": (117649, 663552)}


@pytest.mark.parametrize("name", ["C1", "C2", "C3"])
def test_config_counts_and_orientation(name):
    m = W.make_config(name)
    assert (m.n_nodes, m.n_tets) == COUNTS[name]
    v6 = W.signed_volumes6(m.xyz, m.tets)
    assert np.all(v6 > 0)
    # jitter keeps every tet valid: none inverted relative to the unjittered split
    c = W.CONFIGS[name]
    xyz0, tets0, h, b = W.kuhn_grid(c["lo"], c["hi"], c["cells"])
    assert np.all(W.signed_volumes6(m.xyz, W.orient_positive(xyz0, tets0)) > 0)
    # boundary nodes stay on the box
    assert np.all(m.xyz >= np.array(c["lo"]) - 1e-15) and np.all(m.xyz <= np.array(c["hi"]) + 1e-15)


def test_kuhn_mesh_is_conforming():
    xyz, tets, h, b = W.kuhn_grid((0, 0, 0), (1, 1, 1), (3, 4, 2))
    faces = {}
    for t in tets:
        for f in range(4):
            key = tuple(sorted(int(t[j]) for j in range(4) if j != f))
            faces[key] = faces.get(key, 0) + 1
    counts = np.array(list(faces.values()))
    assert counts.max() == 2
    # boundary faces: 2 triangles per boundary square
    n_bnd = 2 * 2 * (3 * 4 + 4 * 2 + 3 * 2)
    assert np.sum(counts == 1) == n_bnd
    # volumes add up to the box
    assert abs(W.signed_volumes6(xyz, W.orient_positive(xyz, tets)).sum() / 6.0 - 1.0) < 1e-12


def test_jitter_is_seeded():
    a = W.make_config("C1")
    b = W.make_config("C1")
    c = W.make_config("C1", seed=99)
    assert np.array_equal(a.xyz, b.xyz) and not np.array_equal(a.xyz, c.xyz)


def test_fourier_field_is_divergence_free():
    # curl of a potential: central-difference divergence vanishes to O(eps^2)
    rng = np.random.default_rng(1)
    p = rng.uniform(-1, 1, size=(50, 3))
    e = 1e-5
    div = np.zeros(50)
    for c in range(3):
        d = np.zeros(3)
        d[c] = e
        div += (W.field_fourier_curl(p + d, seed=3, normalize=False)[:, c]
                - W.field_fourier_curl(p - d, seed=3, normalize=False)[:, c]) / (2 * e)
    assert np.max(np.abs(div)) < 1e-4
