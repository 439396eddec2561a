"""Benchmark of the layered-media FMM apply on one MI355X.

Workload: the mixed-precision uniform case -- N = M = 100000 sources and
targets in the slabs x in [0,1], y in (0.05,1) / (-0.95,-0.05) of the medium
k = (10, 20, 15) + 0.01i, d = 1; complex64 densities; order 16 on a 7-level
quadtree; FP32 expansions and translations with FP64 sigma tables.  A step is
one complete apply (bounding box, tree build, upward pass, M2L, downward pass,
local evaluation and near field) with all inputs resident in HBM.

Prints one JSON line with the throughput in source-target interactions/s,
the same workload through the plain FP64 FMM, the near-interface workload
(FP64, near field by sweeps), the batched workload (16
instances with their own media, 4 right-hand sides each) as one graph launch
against the FP64 FMM applied instance by instance, the roofline of the
dominant kernel (HIP-event durations of its launches in the timed region,
algorithmic work from the plan's counts) and the FP64 oracle timed on this
host's cores on a bounded sample of targets.

--copy-probe MIB runs only a plain device copy of that size (the calibration
kernel for the HBM byte counters) and exits.
"""
import argparse
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from paper_1902_08250_amd import workloads  # noqa: E402
from paper_1902_08250_amd.prof_summary import source_hash  # noqa: E402

# MI355X published peaks
PEAK = {"fp32": 157.3e12, "fp64": 78.6e12, "hbm": 8.0e12}
# kernel of each timing class on this workload (FP32 expansions, leaf order 16)
KERNEL_NAMES = {"p2m": "k_p2m<float, 16>", "m2m": "k_up<float>", "m2l": "k_m2l_all<float>", "l2l": "k_down<float>",
                "near_sweep": "k_near_sweep<float>", "l2p_near": "k_l2p<float, 16, 1>"}
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic_mixed_uniform_1e5.md")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64 FMM leg")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched leg")
    ap.add_argument("--no-near", action="store_true", help="skip the near-interface leg")
    ap.add_argument("--only-near", action="store_true", help="run only the near-interface leg")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB")
    return ap.parse_args()


def recorded_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed counter summary,
    if it was taken on the current kernel sources (else None)."""
    try:
        text = open(TRAFFIC_FILE).read()
    except OSError:
        return None
    m = re.search(r"source_sha256:\s*([0-9a-f]+)", text)
    if not m or m.group(1) != source_hash():
        return None
    m = re.search(r"^\|\s*%s\s*\|[^\n]*?\|\s*bytes_per_launch=([0-9.eE+]+)" % re.escape(kernel), text, re.M)
    return float(m.group(1)) if m else None


def copy_probe(torch, mib):
    n = mib * (1 << 20) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        torch.mul(a, 1.0, out=b)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe": {"kernel": "elementwise mul by 1 (float32)", "read_bytes": 4 * n,
                                     "write_bytes": 4 * n, "launches": 3}}), flush=True)


def run_gpu(torch, Plan, w, precision, steps, warmup, timing=False, domain=None):
    """Times `steps` applies (the second warm-up apply captures the launch
    sequence as a HIP graph, the timed ones replay it).  With timing, the same
    steps are run again kernel by kernel with HIP start/stop events on every
    kernel launch of the apply's stream, for the per-kernel durations."""
    dt = torch.complex128 if precision == "c128" else torch.complex64
    src = torch.from_numpy(w["src"]).cuda()
    tgt = torch.from_numpy(w["tgt"]).cuda()
    q = torch.from_numpy(w["q"].astype(np.complex128 if precision == "c128" else np.complex64)).cuda()
    u = torch.empty((q.shape[0], tgt.shape[1]), dtype=dt, device="cuda")
    pl = Plan(w["k"], w["d"], order=w["order"], tol=w["tol"] if precision == "c64" else 1e-10, levels=w["levels"])
    if domain:
        pl.set_option("domain", domain)
    for _ in range(max(warmup, 2)):
        pl.apply(src, q, tgt, out=u)
    torch.cuda.synchronize()
    g0 = pl.stats()["graph_applies"]
    t0 = time.perf_counter()
    for _ in range(steps):
        pl.apply(src, q, tgt, out=u)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    st = pl.stats()
    st["graph_applies"] -= g0
    out = u.cpu().numpy()
    if timing:
        pl.set_option("timing", "1")
        pl.apply(src, q, tgt, out=u)
        pl.set_option("timing", "reset")
        t2 = time.perf_counter()
        for _ in range(steps):
            pl.apply(src, q, tgt, out=u)
        torch.cuda.synchronize()
        st_t = pl.stats()
        st_t["ms_per_step_kernel_by_kernel"] = (time.perf_counter() - t2) / steps * 1e3
        st_t["graph_applies"] = st["graph_applies"]
        st = st_t
    return (t1 - t0) / steps, out, st


def roofline(st):
    """Dominant kernel of the timed applies (tree-build group excluded: it is
    many small kernels) against the FP32 vector peak."""
    nap = max(1, st["timed_applies"])
    cand = {k: v for k, v in st["kernel_ms"].items() if k in KERNEL_NAMES and st["kernel_launches"][k] > 0}
    dom = max(cand, key=cand.get)
    ms_apply = cand[dom] / nap
    launches = st["kernel_launches"][dom] / nap
    avg_s = ms_apply / launches * 1e-3
    flops_launch = st["kernel_flops"][dom] / launches
    achieved = flops_launch / avg_s
    kname = KERNEL_NAMES[dom]
    traffic = recorded_traffic(kname)
    return {"kernel": kname, "bound": "alu", "achieved": achieved / 1e12, "peak": PEAK["fp32"] / 1e12,
            "unit": "TFLOP/s", "frac": achieved / PEAK["fp32"], "traffic": traffic,
            "flops_per_launch": flops_launch, "launches_per_apply": launches, "avg_launch_us": avg_s * 1e6,
            "hbm_GBps_if_traffic": (traffic / avg_s / 1e9) if traffic else None}


def batched_leg(torch, steps, warmup):
    from paper_1902_08250_amd.lmfmm import Batch, Plan
    inst = workloads.make_batched()
    inter = float(sum(d["src"].shape[1] * d["tgt"].shape[1] * d["q"].shape[0] for d in inst))
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()  # noqa: E731
    items = [(dev(d["src"]), dev(d["q"]), dev(d["tgt"])) for d in inst]
    t0 = time.perf_counter()
    b = Batch([(d["k"], d["d"]) for d in inst], order_set=(12, 16, 20), tol=1e-6)
    outs = b.apply(items)
    torch.cuda.synchronize()
    t_prep = time.perf_counter() - t0
    for _ in range(warmup):
        b.apply(items, outs=outs)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        b.apply(items, outs=outs)
    torch.cuda.synchronize()
    tb = (time.perf_counter() - t0) / steps
    # plain FP64 FMM, instance after instance
    items64 = [(s, dev(d["q"].astype(np.complex128)), t) for (s, _, t), d in zip(items, inst)]
    plans = [Plan(d["k"], d["d"], order=16, tol=1e-10) for d in inst]
    outs64 = [p.apply(*it) for p, it in zip(plans, items64)]
    torch.cuda.synchronize()
    n64 = max(2, steps // 4)
    t0 = time.perf_counter()
    for _ in range(n64):
        for p, it, o in zip(plans, items64, outs64):
            p.apply(*it, out=o)
    torch.cuda.synchronize()
    t64 = (time.perf_counter() - t0) / n64
    errs = [float(np.linalg.norm(o.cpu().numpy().astype(np.complex128) - r.cpu().numpy()) /
                  np.linalg.norm(r.cpu().numpy())) for o, r in zip(outs, outs64)]
    return {"workload": "batched: 16 instances, N log-uniform in [1e3, 2e5], own media, 4 RHS each, c64",
            "value": inter / tb, "unit": "interactions/s", "ms_per_step": tb * 1e3,
            "prepare_s": t_prep, "choices": b.choices(),
            "fp64_fmm_sequential": {"value": inter / t64, "ms_per_step": t64 * 1e3},
            "speedup_vs_fp64_sequential": t64 / tb, "rel_l2_max_vs_fp64_fmm": max(errs)}


def near_leg(torch, Plan, steps, warmup):
    """The near-interface workload (2e5 sources and targets within 1e-3 of
    the interface, medium k = (40, 60, 50) + 0.01i, d = 0.5, FP64, order 20,
    12 levels): the near field is the x-ordered sweep of the row-0 leaves."""
    w = workloads.make(2)
    inter = float(w["n_src"]) * w["n_tgt"] * w["nrhs"]
    n = max(3, steps // 4)
    t, _, st = run_gpu(torch, Plan, w, "c128", n, warmup, timing=True)
    nap = max(1, st["timed_applies"])
    sweep_ms = st["kernel_ms"]["near_sweep"] / nap
    return {"workload": w["name"], "n_src": w["n_src"], "n_tgt": w["n_tgt"], "order": w["order"],
            "levels": w["levels"], "tol": 1e-10, "dtype": "f64", "steps": n, "value": inter / t,
            "unit": "interactions/s", "ms_per_step": t * 1e3,
            "kernel_ms_per_apply": {k: v / nap for k, v in st["kernel_ms"].items() if v > 0},
            "near_sweep": {"kernel": "k_near_sweep<double, 1>", "ms_per_launch": sweep_ms,
                           "nodes": st["near_nodes_mid"] + 2 * st["near_nodes_ray"]}}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported "
              "(the multi-GPU sharding is a design, not a build)", file=sys.stderr)
        sys.exit(2)
    import torch
    if args.copy_probe:
        copy_probe(torch, args.copy_probe)
        return
    from paper_1902_08250_amd.lmfmm import Plan
    if args.only_near:
        print(json.dumps({"near_interface": near_leg(torch, Plan, args.steps, args.warmup)}), flush=True)
        return

    w = workloads.make(1)
    n_src, n_tgt, nrhs = w["n_src"], w["n_tgt"], w["nrhs"]
    inter = float(n_src) * n_tgt * nrhs

    print(f"[bench] workload {w['name']}: warmup {args.warmup}, steps {args.steps}", file=sys.stderr, flush=True)
    t_mixed, u_mixed, st = run_gpu(torch, Plan, w, "c64", args.steps, args.warmup, timing=True)
    print(f"[bench] mixed: {t_mixed * 1e3:.3f} ms/step", file=sys.stderr, flush=True)
    nap = max(1, st["timed_applies"])
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
        "kernel_ms_per_apply": {k: v / nap for k, v in st["kernel_ms"].items() if v > 0},
        "ms_per_step_kernel_by_kernel_with_events": st["ms_per_step_kernel_by_kernel"],
        "kernel_launches_per_apply": {k: v / nap for k, v in st["kernel_launches"].items() if v > 0},
        "m2l_pairs": st["m2l_pairs"],
        "graph_applies_in_timed_region": st["graph_applies"],
        "roofline": roofline(st),
    }
    # the same applies with the domain given up front: no bounding-box readback,
    # so consecutive applies are queued without a host round trip in between
    t_dom, u_dom, _ = run_gpu(torch, Plan, w, "c64", args.steps, args.warmup, domain="0,1,1,-0.95")
    out["fixed_domain"] = {"value": inter / t_dom, "ms_per_step": t_dom * 1e3, "domain": "x in [0,1], y_s < 1, y_t > -0.95",
                           "max_abs_diff_vs_auto": float(np.max(np.abs(u_dom - u_mixed)))}
    if not args.no_fp64:
        t64, u64, _ = run_gpu(torch, Plan, w, "c128", max(3, args.steps // 4), 1)
        print(f"[bench] fp64: {t64 * 1e3:.3f} ms/step", file=sys.stderr, flush=True)
        out["fp64_fmm"] = {"value": inter / t64, "ms_per_step": t64 * 1e3}
        out["mixed_over_fp64"] = t64 / t_mixed
        out["rel_l2_mixed_vs_fp64_fmm"] = float(np.linalg.norm(u_mixed - u64) / np.linalg.norm(u64))
    if not args.no_near:
        out["near_interface"] = near_leg(torch, Plan, args.steps, args.warmup)
        print(f"[bench] near-interface: {out['near_interface']['ms_per_step']:.3f} ms/step", file=sys.stderr,
              flush=True)
    if not args.no_batched:
        out["batched"] = batched_leg(torch, args.steps, args.warmup)
        print(f"[bench] batched: {out['batched']['ms_per_step']:.3f} ms/step", file=sys.stderr, flush=True)

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
        if not args.no_fp64:
            out["rel_l2_fp64_vs_oracle_sample"] = float(np.linalg.norm(u64[:, sel] - ref) / np.linalg.norm(ref))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
