"""Equal-accuracy study of the rule policies on a full-size workload (not a
pytest module; run it by name on a GPU machine):

    python tests/study_equal_accuracy.py [C2] [24] [out.json]

Probe nodes: seeded interior nodes of the workload where |w| is above its
60th percentile.  Exact reference at each: the cone-decomposition integral
of every tet whose centroid is within four mean edge lengths (order-16
brute force, oracle/references.py), the 11-point rule beyond (at most a few
1e-7 of the result there).  For each policy: rel-L2 error at the probes and
the median device time of one evaluation of the whole mesh."""
import json
import os
import sys
import time
from multiprocessing import Pool

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))

import oracle  # noqa: E402
import workloads as W  # noqa: E402
from oracle import references as R  # noqa: E402

NAME = sys.argv[1] if len(sys.argv) > 1 else "C2"
NPROBE = int(sys.argv[2]) if len(sys.argv) > 2 else 24
OUT = sys.argv[3] if len(sys.argv) > 3 else None

M = W.make_config(NAME)
HB = oracle.mean_edge(M.xyz, M.tets)
CEN = M.xyz[M.tets].mean(axis=1)


def exact_at(i):
    d = np.linalg.norm(CEN - M.xyz[i], axis=1)
    near, far = np.nonzero(d < 4 * HB)[0], np.nonzero(d >= 4 * HB)[0]
    e = np.zeros(3)
    for t in near:
        e += R.tet_cone_brute_force(M.xyz[i], M.xyz[M.tets[t]], M.omega[M.tets[t]], order=16)
    e += oracle.evaluate(M.xyz, M.omega, M.tets[far], targets=[i],
                         pair_rules=np.full((1, far.size), 2, np.int8))[0]
    return e


def main():
    rng = np.random.default_rng(7)
    wn = np.linalg.norm(M.omega, axis=1)
    cand = np.nonzero((~M.boundary) & (wn > np.quantile(wn, 0.6)))[0]
    tg = rng.choice(cand, NPROBE, replace=False)
    t0 = time.time()
    with Pool(min(16, os.cpu_count() or 1)) as pool:
        exact = np.array(pool.map(exact_at, list(tg)))
    print(f"exact references at {len(tg)} probes: {time.time() - t0:.1f} s", flush=True)

    import paper_0712_1695_amd as bs

    blob = json.load(open(os.path.join(HERE, "golden", "selector_blob.json")))
    bits = np.array(blob["blob_bf16_bits"], dtype=np.uint16)
    fixed = [(2, 4, 8, 16), (1.5, 4, 8, 16), (1.0, 4, 8, 16), (2.5, 4, 8, 16), (2, 6, 8, 16), (2, 4, 8, 24),
             (2, 4, 8, 32), (2, 4, 8, 48), (1.5, 4, 8, 24), (1.5, 4, 8, 32)]
    configs = [dict(kind=bs.BS_POLICY_FIXED, near_cut=a, d_g11=b, d_g4=c, n_phi=nl, n_theta=nl)
               for a, b, c, nl in fixed]
    configs += [dict(kind=bs.BS_POLICY_LEARNED, mlp_bf16=bits, conf_min=c, n_phi=nl, n_theta=nl)
                for c, nl in ((0.9, 16), (0.8, 16), (0.95, 16), (0.9, 24))]
    h = bs.bs_mesh_upload(M.xyz, M.omega, M.tets)
    rows = []
    try:
        for pol in configs:
            bs.bs_set_policy(h, **pol)
            for _ in range(2):
                bs.bs_eval_velocity(h)
            ts = []
            for _ in range(5):
                v, st = bs.bs_eval_velocity(h, stats=True)
                ts.append(st["t_eval_s"])
            row = {k: v2 for k, v2 in pol.items() if k != "mlp_bf16"}
            row["kind"] = "learned" if pol["kind"] == bs.BS_POLICY_LEARNED else "fixed"
            row.update(err=float(np.linalg.norm(v[tg] - exact) / np.linalg.norm(exact)),
                       ms=1e3 * float(np.median(ts)), rt_pairs=int(st["pairs_by_rule"][3]))
            rows.append(row)
            print(json.dumps(row), flush=True)
    finally:
        bs.bs_mesh_free(h)
    if OUT:
        json.dump(dict(workload=NAME, probes=int(len(tg)), rows=rows), open(OUT, "w"), indent=1)


if __name__ == "__main__":
    main()
