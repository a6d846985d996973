"""Write tests/golden/c5_heun_step1.json: one Heun step of the two-ring
workload (80^3 Kuhn cells, 531,441 nodes, 3,072,000 tetrahedra) computed by
the FP64 oracle alone, at a seeded sample of nodes.

    python tests/golden/make_c5_heun_reference.py SCRATCH_DIR [OUT.json]

Heun (RK2) with dt = 0.005, connectivity and nodal vorticity kept:
    v1 = v(x);  x* = x + dt v1;  v2 = v(x*);  x1 = x + dt/2 (v1 + v2).
v1 is needed at every node (x* moves every node), so the oracle evaluates
the whole mesh once (about three hours on eight host threads); the chunks
are checkpointed in SCRATCH_DIR so that an interrupted run resumes.  v2 and
x1 are then evaluated at the sample only.  Policy: the fixed distance rule
(ray tracing within 2 mean edge lengths, 11-point rule within 4, 4-point
within 8, else 1-point), 16 x 16 lines.  Nothing here runs the GPU library.
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import workloads as W  # noqa: E402

DT = 0.005
CHUNK = 4096
N_SAMPLE = 256


def sample_nodes(m):
    """128 interior nodes drawn among the 5% of largest |omega| (the ring
    cores) and 128 drawn uniformly among all interior nodes, seed 5."""
    rng = np.random.default_rng(5)
    interior = np.nonzero(~m.boundary)[0]
    wn = np.linalg.norm(m.omega[interior], axis=1)
    core = interior[wn >= np.quantile(wn, 0.95)]
    a = rng.choice(core, N_SAMPLE // 2, replace=False)
    rest = np.setdiff1d(interior, a)
    b = rng.choice(rest, N_SAMPLE - N_SAMPLE // 2, replace=False)
    return np.sort(np.concatenate([a, b]))


def main():
    scratch = sys.argv[1]
    out = sys.argv[2] if len(sys.argv) > 2 else os.path.join(HERE, "c5_heun_step1.json")
    os.makedirs(scratch, exist_ok=True)
    m = W.make_config("C5")
    pol = oracle.make_policy("fixed")
    n = m.n_nodes
    v1 = np.zeros((n, 3))
    t0 = time.time()
    for c0 in range(0, n, CHUNK):
        path = os.path.join(scratch, f"v1_{c0:07d}.npy")
        tg = np.arange(c0, min(n, c0 + CHUNK))
        if os.path.exists(path):
            v1[tg] = np.load(path)
            continue
        v = oracle.evaluate(m.xyz, m.omega, m.tets, pol, targets=tg)
        np.save(path + ".tmp.npy", v)
        os.replace(path + ".tmp.npy", path)
        v1[tg] = v
        print(f"v1 nodes {c0}..{tg[-1]} of {n}: {time.time() - t0:.0f} s", flush=True)
    xs = m.xyz + DT * v1
    smp = sample_nodes(m)
    v2 = oracle.evaluate(xs, m.omega, m.tets, pol, targets=smp)
    x1 = m.xyz[smp] + 0.5 * DT * (v1[smp] + v2)
    doc = {
        "what": "one Heun step of the two-ring workload by the FP64 oracle at sampled nodes",
        "workload": "C5: two coaxial rings, [-1.5,1.5]^3, 80^3 Kuhn cells, jitter 0.2 h, seed 5",
        "policy": "fixed rule (RT < 2 hbar, G11 < 4, G4 < 8, else G1), 16 x 16 lines, FP64",
        "dt": DT,
        "script": "tests/golden/make_c5_heun_reference.py",
        "nodes": smp.tolist(),
        "v1": v1[smp].tolist(),
        "v2": v2.tolist(),
        "x1": x1.tolist(),
        "oracle_threads": oracle.num_threads(),
        "seconds": time.time() - t0,
    }
    with open(out, "w") as f:
        json.dump(doc, f)
    print(f"wrote {out}", flush=True)


if __name__ == "__main__":
    main()
