"""Benchmark: node-tet pair evaluations per second on one MI355X.

One step = one bs_eval_velocity on the vortex-ring workload (a
[-1.5,1.5]^2 x [-0.5,0.5] box, 64 x 64 x 22 Kuhn-split cells: 97,175 nodes,
540,672 tetrahedra, jitter 0.15 h; Gaussian-core ring, radius 1, sigma 0.1;
fixed distance rule with ray tracing below 2 mean edge lengths, 16 x 16
angular rule, FP32 with compensated accumulation).  Inputs are resident in
HBM before the timed region; the output goes to device memory.

Prints one JSON line (see the keys below).  The timed steps run the band
and ray-tracing kernels beside the far field (library streams); a second
pass of the same steps with every kernel on one stream gives each kernel's
own duration (HIP events recorded on its launch stream inside the library),
from which the roofline objects of the three kernels are computed
("roofline" is the longest of them, "roofline_kernels" lists all).  cpu_baseline
times the FP64 oracle on a bounded sample of nodes (all tetrahedra) on the
host's cores.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

FP32_PEAK_TFLOPS = 157.3  # MI355X FP32 vector: 256 CUs x 2.4 GHz x 256 flop/clk
FLOPS_PER_POINT = 26.0     # one Gauss point: 3 sub, |r|^2 (5), rsqrt (1), r^-3 (2), W x r / r^3 + acc (15)


def algorithmic_flops(st, nm):
    """Method flop count of one evaluation: 26 per Gauss point, ray tracing
    9 per pair + 7 per line (the precheck) + 156 per line that hits."""
    g1, g4, g11, rt = st["pairs_by_rule"]
    return (FLOPS_PER_POINT * (g1 + 4 * g4 + 11 * g11) + rt * (9.0 + 7.0 * nm) + 156.0 * st["rt_hit_lines"])


WORKLOAD_TEXT = {
    "C1": "Gaussian swirl, [-1,1]^3, 10^3 Kuhn cells",
    "C2": "vortex ring, [-1.5,1.5]^2 x [-0.5,0.5], 64x64x22 Kuhn cells",
    "C3": "random Fourier curl field, [-1,1]^3, 48^3 Kuhn cells",
    "C5": "two coaxial rings, [-1.5,1.5]^3, 80^3 Kuhn cells",
}


def measured_traffic(kernel, workload, precision):
    """HBM bytes per launch of `kernel` from the committed counter summary,
    or None when the kernel source has changed since the counters were
    taken (the summary records the sha256 of that source) or the run is not
    the profiled configuration."""
    import hashlib

    if workload != "C2" or precision != 1:
        return None
    path = os.path.join(ROOT, "profiles", "bs_eval_velocity_C2_hbm_traffic.md")
    src = os.path.join(ROOT, "paper_0712_1695_amd", "csrc", "bs_kernels.hip")
    try:
        lines = open(path).read().split("\n")
        sha = hashlib.sha256(open(src, "rb").read()).hexdigest()
    except OSError:
        return None
    for ln in lines:
        f = ln.split()
        if len(f) == 4 and f[0] == "traffic" and f[1] == kernel and f[3] == sha:
            return float(f[2])
    return None


def copy_calibration(mib):
    """A plain device-to-device copy of a known size, so that the HBM byte
    counters of a profiler can be scaled: it reads and writes mib MiB."""
    import torch

    n = mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": n * 4, "copy_bytes_written": n * 4}), flush=True)


def cpu_baseline(mesh, target_seconds=15.0):
    import oracle

    pol = oracle.make_policy("fixed")
    rng = np.random.default_rng(123)
    k = 8
    while True:
        tg = rng.choice(mesh.n_nodes, size=k, replace=False)
        t0 = time.perf_counter()
        oracle.evaluate(mesh.xyz, mesh.omega, mesh.tets, pol, targets=tg)
        dt = time.perf_counter() - t0
        if dt >= target_seconds / 2 or k >= mesh.n_nodes // 2:
            break
        k = min(mesh.n_nodes // 2, int(k * max(2.0, target_seconds / max(dt, 1e-3))))
    pairs = k * mesh.n_tets
    return {"value": pairs / dt, "unit": "pairs/s", "cores": oracle.num_threads(), "kind": "oracle",
            "sample": f"{k} random nodes x all {mesh.n_tets} tets of the same workload (FP64, fixed rule), "
                      f"{dt:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="C2")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--precision", type=int, default=1)
    ap.add_argument("--no-learned", action="store_true", help="skip the learned-policy leg")
    ap.add_argument("--serial", action="store_true",
                    help="time the steps with every kernel on one stream too (for per-kernel profiles)")
    ap.add_argument("--valu-far", action="store_true",
                    help="far field on the vector ALUs instead of the matrix cores (comparison)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain copy of MIB MiB (profiler byte-counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (--gpus {args.gpus} requested); multi-GPU sharding is not built",
              file=sys.stderr)
        sys.exit(2)

    if args.copy_calibration:
        copy_calibration(args.copy_calibration)
        return

    import torch

    import paper_0712_1695_amd as bs
    import workloads as W

    torch.cuda.set_device(0)
    dev = torch.device("cuda", 0)
    mesh = W.make_config(args.workload)
    xyz = torch.tensor(mesh.xyz, device=dev)
    om = torch.tensor(mesh.omega, device=dev)
    tets = torch.tensor(mesh.tets, device=dev)
    h = bs.bs_mesh_upload(xyz, om, tets)
    nm = 16 * 16
    bs.bs_set_policy(h, kind=bs.BS_POLICY_FIXED, n_phi=16, n_theta=16, precision=args.precision)
    out = torch.empty((mesh.n_nodes, 3), dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream()

    for _ in range(args.warmup):
        bs.bs_eval_velocity(h, out=out, valu_far=args.valu_far)
    torch.cuda.synchronize()

    # the timed steps: band and ray tracing run beside the far field
    t0 = time.perf_counter()
    for _ in range(args.steps):
        bs.bs_eval_velocity(h, out=out, valu_far=args.valu_far, serial=args.serial)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    _, stats = bs.bs_eval_velocity(h, out=out, stats=True, valu_far=args.valu_far, serial=args.serial)
    # the same steps with every kernel on one stream: each kernel's own
    # duration (HIP events on its launch stream) for the roofline
    kern = np.zeros(4)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        _, st_s = bs.bs_eval_velocity(h, out=out, stats=True, valu_far=args.valu_far, serial=True)
        kern += np.array(st_s["t_kernel_s"])
    torch.cuda.synchronize()
    wall_serial = time.perf_counter() - t0
    kern /= max(args.steps, 1)

    pairs = mesh.n_nodes * mesh.n_tets
    ms = wall / args.steps * 1e3
    value = pairs / (wall / args.steps)

    learned = None
    if not args.no_learned:
        # the selector is trained on the GPU by the library's own kernels
        # (outside the timed region), on pairs of two smaller meshes, then
        # the same evaluation is timed with the learned policy
        from paper_0712_1695_amd import selector

        train_meshes = [W.make_config("C1"), W.make_config("C2", scale=(32, 32, 11))]
        blob, info = selector.train([(t.xyz, t.omega, t.tets) for t in train_meshes])
        conf_min = 0.9
        bs.bs_set_policy(h, kind=bs.BS_POLICY_LEARNED, n_phi=16, n_theta=16, precision=args.precision,
                         mlp_bf16=blob, conf_min=conf_min)
        for _ in range(args.warmup):
            bs.bs_eval_velocity(h, out=out, valu_far=args.valu_far)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            bs.bs_eval_velocity(h, out=out, valu_far=args.valu_far)
        torch.cuda.synchronize()
        wall_l = time.perf_counter() - t0
        kl = np.zeros(4)
        for _ in range(args.steps):
            _, st_l = bs.bs_eval_velocity(h, out=out, stats=True, valu_far=args.valu_far, serial=True)
            kl += np.array(st_l["t_kernel_s"])
        kl /= max(args.steps, 1)
        value_l = pairs / (wall_l / args.steps)
        learned = {"value": value_l, "unit": "pairs/s", "ms_per_step": wall_l / args.steps * 1e3,
                   "vs_fixed": value_l / value, "conf_min": conf_min, "pairs_by_rule": st_l["pairs_by_rule"],
                   "rt_hit_lines": st_l["rt_hit_lines"],
                   "kernel_ms_serial": {"far": kl[0] * 1e3, "band": kl[1] * 1e3, "rt": kl[2] * 1e3,
                                        "sum": kl[3] * 1e3},
                   "selector": {**info, "trained_on": [t.name for t in train_meshes]}}
    flops = algorithmic_flops(stats, nm)
    g1, g4, g11, rtp = stats["pairs_by_rule"]
    far_name = "k_gauss_all" if (args.valu_far or args.precision == 2) else "k_far_mfma"
    band_name = "k_band" if far_name == "k_gauss_all" else "k_band_piece"
    measured = "kernel alone: the serial pass (every kernel on one stream), HIP events on its stream"

    def roof_entry(name, what, bound, kflops, t):
        return {"kernel": f"{name} ({what})", "bound": bound, "achieved": kflops / t / 1e12,
                "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": kflops / t / 1e12 / FP32_PEAK_TFLOPS,
                "traffic": measured_traffic(name, args.workload, args.precision),
                "traffic_unit": "bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
                "avg_duration_ms": t * 1e3, "measured": measured}

    kernels = [
        roof_entry(far_name, "far field, 1-point rule on every pair, vector ALUs" if far_name == "k_gauss_all"
                   else "far field, the G1 pairs, FP32 matrix-core contractions",
                   "alu" if far_name == "k_gauss_all" else "mfma", FLOPS_PER_POINT * g1, kern[0]),
        roof_entry(band_name, "the G4 and G11 pairs, vector ALUs, lane = node" +
                   ("" if band_name == "k_band" else ", row pieces staged in LDS"), "alu",
                   FLOPS_PER_POINT * (4 * g4 + 11 * g11), kern[1]),
        roof_entry("k_rt_walk", "ray tracing by walking face neighbours; the method's flops of its pairs", "alu",
                   rtp * (9.0 + 7.0 * nm) + 156.0 * stats["rt_hit_lines"], kern[2]),
    ]
    # the dominant kernel: the longest one alone
    roof = dict(max(kernels, key=lambda r: r["avg_duration_ms"]))
    line = {
        "metric": "node-tet pair evals/s (+ % FP32 peak)",
        "value": value,
        "unit": "pairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": f"{args.workload}: {WORKLOAD_TEXT.get(args.workload, mesh.name)}, {mesh.n_nodes} nodes x "
                        f"{mesh.n_tets} tets, fixed rule (RT < 2 hbar, G11 < 4, G4 < 8, else G1), 16x16 lines, "
                        f"{['fp32 naive', 'fp32 compensated', 'fp64 accumulation'][args.precision]}",
            "pairs_per_step": pairs,
            "pairs_by_rule": stats["pairs_by_rule"],
            "rt_hit_lines": stats["rt_hit_lines"],
            "algorithmic_tflop_per_step": flops / 1e12,
            "path_fp32_peak_frac": flops / (wall / args.steps) / 1e12 / FP32_PEAK_TFLOPS,
            "ms_per_step_serial": wall_serial / args.steps * 1e3,
            "kernel_ms_serial": {"far": kern[0] * 1e3, "band": kern[1] * 1e3, "rt": kern[2] * 1e3,
                                 "sum": kern[3] * 1e3},
        },
        "roofline": roof,
        "roofline_kernels": kernels,
    }
    if learned is not None:
        line["learned"] = learned
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(mesh)
    bs.bs_mesh_free(h)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
