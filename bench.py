"""Benchmark of the layered-media FMM apply on one MI355X.

Workload: the mixed-precision uniform case -- N = M = 100000 sources and
targets in the slabs x in [0,1], y in (0.05,1) / (-0.95,-0.05) of the medium
k = (10, 20, 15) + 0.01i, d = 1; complex64 densities; order 16 on a 7-level
quadtree; FP32 expansions and translations with FP64 sigma tables.  A step is
one complete apply (bounding box, tree build, upward pass, M2L, downward pass,
local evaluation and near field) with all inputs resident in HBM.

Prints one JSON line with the throughput in source-target interactions/s,
the same workload through the plain FP64 FMM, the roofline of the dominant
kernel (HIP-event durations of its launches in the timed region) and the FP64
oracle timed on this host's cores on a bounded sample of targets.
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from paper_1902_08250_amd import workloads  # noqa: E402

PEAK = {"fp32": 157.3e12, "fp64": 78.6e12, "hbm": 8.0e12}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    return ap.parse_args()


def p2m_flops_per_point(P, kr):
    """Arithmetic of the scaled-basis evaluation and accumulation of one point
    (per right-hand side for the accumulation):
      backward ratio recurrence, N = P + 16 + floor(1.2 |k r|) steps of
      z^2 t (6) + subtract (1) + complex reciprocal (6) + normalisation
      update every other step (6 per step)  -> 19 flops per step;
      forward products: 2 q t (2) + f*up (6) + v*... (6), twice -> 26 per order;
      accumulation: 2P+1 complex multiply-adds (8 flops each)."""
    N = P + 16 + int(1.2 * kr)
    return 19 * N + 26 * P + 8 * (2 * P + 1)


def run_gpu(torch, Plan, w, precision, steps, warmup, timing=False):
    dt = torch.complex128 if precision == "c128" else torch.complex64
    src = torch.from_numpy(w["src"]).cuda()
    tgt = torch.from_numpy(w["tgt"]).cuda()
    q = torch.from_numpy(w["q"].astype(np.complex128 if precision == "c128" else np.complex64)).cuda()
    u = torch.empty((q.shape[0], tgt.shape[1]), dtype=dt, device="cuda")
    pl = Plan(w["k"], w["d"], order=w["order"], tol=w["tol"] if precision == "c64" else 1e-10, levels=w["levels"])
    for _ in range(warmup):
        pl.apply(src, q, tgt, out=u)
    torch.cuda.synchronize()
    if timing:
        pl.set_option("timing", "1")
        pl.set_option("timing", "reset")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        pl.apply(src, q, tgt, out=u)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    st = pl.stats()
    return (t1 - t0) / steps, u.cpu().numpy(), st, pl


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported "
              "(the multi-GPU sharding is a design, not a build)", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_1902_08250_amd.lmfmm import Plan

    w = workloads.make(1)
    n_src, n_tgt, nrhs = w["n_src"], w["n_tgt"], w["nrhs"]
    inter = float(n_src) * n_tgt * nrhs

    print(f"[bench] workload {w['name']}: warmup {args.warmup}, steps {args.steps}", file=sys.stderr, flush=True)
    t_mixed, u_mixed, st, pl = run_gpu(torch, Plan, w, "c64", args.steps, args.warmup, timing=True)
    print(f"[bench] mixed: {t_mixed * 1e3:.3f} ms/step", file=sys.stderr, flush=True)
    t64, u64, st64, _ = run_gpu(torch, Plan, w, "c128", max(3, args.steps // 4), 1)
    print(f"[bench] fp64: {t64 * 1e3:.3f} ms/step", file=sys.stderr, flush=True)
    rel_mixed_fp64 = float(np.linalg.norm(u_mixed - u64) / np.linalg.norm(u64))

    # roofline of the dominant stage kernel (single-launch stages measured by events)
    names = ["tree", "p2m", "m2m", "m2l_l2l", "l2p_near"]
    stage_ms = st["stage_ms"]
    nap = max(1, st["timed_applies"])
    per_apply = [m / nap for m in stage_ms]
    dom = int(np.argmax(per_apply))
    L = st["levels"]
    P_leaf = st["order"][L]
    wL = st["root_width"] / 2 ** L
    kr = abs(w["k"][1]) * wL / math.sqrt(2)
    launches = max(1, st["stage_launches"][dom] // nap)
    avg_launch_s = per_apply[dom] / launches * 1e-3
    if names[dom] in ("p2m", "l2p_near"):
        flops = p2m_flops_per_point(P_leaf, kr) * (n_src if names[dom] == "p2m" else n_tgt)
        achieved = flops / avg_launch_s
        roof = {"kernel": "k_p2m" if names[dom] == "p2m" else "k_l2p_near", "bound": "alu",
                "achieved": achieved / 1e12, "peak": PEAK["fp32"] / 1e12, "unit": "TFLOP/s",
                "frac": achieved / PEAK["fp32"], "traffic": None,
                "avg_launch_us": avg_launch_s * 1e6}
    else:
        roof = {"kernel": names[dom], "bound": "alu", "achieved": None, "peak": PEAK["fp32"] / 1e12,
                "unit": "TFLOP/s", "frac": None, "traffic": None, "avg_launch_us": avg_launch_s * 1e6}

    out = {
        "metric": "source-target interactions/s at stated rel-l2 err; mixed+batched vs FP64 FMM",
        "value": inter / t_mixed,
        "unit": "interactions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": t_mixed * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": w["name"], "n_src": n_src, "n_tgt": n_tgt, "nrhs": nrhs, "order": w["order"],
                   "levels": w["levels"], "tol": w["tol"], "orders_by_level": st["order"],
                   "medium": "k=(10,20,15)+0.01i, d=1"},
        "fp64_fmm": {"value": inter / t64, "ms_per_step": t64 * 1e3},
        "mixed_over_fp64": t64 / t_mixed,
        "rel_l2_mixed_vs_fp64_fmm": rel_mixed_fp64,
        "stage_ms_per_apply": dict(zip(names, per_apply)),
        "roofline": roof,
    }

    if not args.no_cpu:
        import oracle
        oracle.build(force=False)
        cores = oracle.max_threads()
        rng = np.random.default_rng(123)
        # size the sample to about cpu_seconds of oracle work
        t0 = time.perf_counter()
        oracle.apply(w["src"], w["q"].astype(np.complex128), w["tgt"][:, :cores], w["k"], w["d"])
        t_probe = time.perf_counter() - t0
        n_s = max(cores, int(cores * args.cpu_seconds / max(t_probe, 1e-3)))
        n_s = min(n_s, n_tgt)
        sel = np.sort(rng.choice(n_tgt, n_s, replace=False))
        t0 = time.perf_counter()
        ref = oracle.apply(w["src"], w["q"].astype(np.complex128), w["tgt"][:, sel], w["k"], w["d"])
        t_cpu = time.perf_counter() - t0
        rate = float(n_s) * n_src * nrhs / t_cpu
        out["cpu_baseline"] = {"value": rate, "unit": "interactions/s", "cores": cores, "kind": "oracle",
                               "sample": f"{n_s} seeded targets x {n_src} sources ({t_cpu:.1f} s)"}
        out["rel_l2_mixed_vs_oracle_sample"] = float(np.linalg.norm(u_mixed[:, sel] - ref) / np.linalg.norm(ref))
        out["rel_l2_fp64_vs_oracle_sample"] = float(np.linalg.norm(u64[:, sel] - ref) / np.linalg.norm(ref))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
