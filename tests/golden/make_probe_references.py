"""Write tests/golden/probe_exact_<NAME>.json: the exact Biot-Savart velocity
of the piecewise-linear vorticity at seeded probe nodes of a workload, for
the accuracy legs of the benchmark and the equal-accuracy test.

    python tests/golden/make_probe_references.py C2 C3 C5

Probes: seeded (seed 7) interior nodes where |omega| exceeds its 60th
percentile (the vortex cores, where the near field matters most).  Exact
value at a probe x (test infrastructure only, oracle/ code):
  - every tetrahedron whose centroid lies within 4 mean edge lengths of x:
    the signed cone decomposition from x with the radial integral exact and
    an order-16 collapsed Gauss rule on each face (references.py);
  - every other tetrahedron: the 11-point (degree 4) rule, whose error there
    is a few 1e-7 of the result at most.
The second part is the oracle's 11-point sum over all tetrahedra minus the
same rule over the near ones.
"""
import json
import os
import sys
import time
from multiprocessing import Pool

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import workloads as W  # noqa: E402
from oracle import references as R  # noqa: E402

N_PROBES = {"C2": 24, "C3": 24, "C5": 32}
NEAR = 4.0
ORDER = 16

_M = None


def _near_part(args):
    """Cone decomposition minus the 11-point rule over the near tets of one
    probe."""
    i, near = args
    m = _M
    x = m.xyz[i]
    e = np.zeros(3)
    for t in near:
        tv, tw = m.xyz[m.tets[t]], m.omega[m.tets[t]]
        e += R.tet_cone_brute_force(x, tv, tw, order=ORDER) - oracle.pair(x, tv, tw, oracle.RULE_G11)
    return e


def probes(m, k):
    rng = np.random.default_rng(7)
    wn = np.linalg.norm(m.omega, axis=1)
    cand = np.nonzero((~m.boundary) & (wn > np.quantile(wn, 0.6)))[0]
    return np.sort(rng.choice(cand, k, replace=False))


def main():
    global _M
    names = sys.argv[1:] or ["C2", "C3", "C5"]
    for name in names:
        t0 = time.time()
        m = W.make_config(name)
        _M = m
        tg = probes(m, N_PROBES[name])
        hb = oracle.mean_edge(m.xyz, m.tets)
        cen = m.xyz[m.tets].mean(axis=1)
        g11_all = oracle.evaluate(m.xyz, m.omega, m.tets, oracle.make_policy("gauss_only", gauss_rule=oracle.RULE_G11),
                                  targets=tg)
        jobs = []
        for i in tg:
            d = np.linalg.norm(cen - m.xyz[i], axis=1)
            jobs.append((int(i), np.nonzero(d < NEAR * hb)[0]))
        with Pool(min(8, os.cpu_count() or 1)) as pool:
            corr = np.array(pool.map(_near_part, jobs))
        exact = g11_all + corr
        doc = {
            "what": "exact velocity of the piecewise-linear vorticity at probe nodes",
            "workload": name,
            "n_nodes": m.n_nodes,
            "n_tets": m.n_tets,
            "recipe": f"cone decomposition (order {ORDER}) within {NEAR} hbar of the probe, 11-point rule beyond",
            "script": "tests/golden/make_probe_references.py",
            "hbar": hb,
            "nodes": tg.tolist(),
            "near_tets": [int(len(j[1])) for j in jobs],
            "velocity": exact.tolist(),
        }
        out = os.path.join(HERE, f"probe_exact_{name}.json")
        with open(out, "w") as f:
            json.dump(doc, f)
        print(f"{name}: {len(tg)} probes, {time.time() - t0:.1f} s -> {out}", flush=True)


if __name__ == "__main__":
    main()
