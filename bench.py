"""Benchmark of the layered-media FMM on one MI355X.

Headline workload (the metric's "mixed + batched"): 16 problem instances with
their own three-layer media (k1 in [5,30], k2 in [10,60], k3 in [5,40], each
+0.01i; d in [0.5, 2]) and log-uniform sizes N = M in [1e3, 2e5], 4 complex64
right-hand sides each, applied as one batch: every stage of all instances is
one merged launch, the sequence replayed as one HIP graph, each instance's
order floor (from {12, 16, 20}) and levels autotuned, tolerance 1e-6.  A step
is one batched apply of all instances (tree build, upward pass, M2L, downward
pass, near field, local evaluation) with every input resident in HBM.
`value` = sum_i N_i M_i nrhs / time per step.

Beside it, on one JSON line:
  * the same batch through the FP64 path (complex128, tol 1e-10, its own
    autotuned choices) as one merged graph: the like-for-like FP64 FMM; and
    the FP64 plans applied instance after instance, for context;
  * errors against the oracle's stored samples of every instance;
  * the roofline of the dominant kernel class of the batched apply (event
    durations of its merged launches, algorithmic flops from the plans'
    counts) and, for the other legs, of theirs;
  * the mixed uniform workload (1e5 x 1e5, one right-hand side, order 16,
    7 levels) with a cold apply (translation tables built in the call);
  * the near-interface workload (2e5 x 2e5 within 1e-3 of the interface,
    FP64) with the roofline of its near-field sweep;
  * the FP64 oracle timed on this host's cores on a bounded sample.

--copy-probe MIB runs only a plain device copy of that size (the calibration
kernel for the HBM byte counters) and exits.
"""
import argparse
import json
import os
import re
import sys
import tempfile
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from paper_1902_08250_amd import workloads  # noqa: E402
from paper_1902_08250_amd.prof_summary import source_hash  # noqa: E402

# MI355X published peaks
PEAK = {"fp32": 157.3e12, "fp64": 78.6e12, "hbm": 8.0e12}
GOLD = os.path.join(ROOT, "tests", "golden")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic_batched_16x4.md")
UNIFORM_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic_mixed_uniform_1e5.md")
# algorithmic FP64 flops of the near-field sweep per (point, node, direction):
# one complex exponential (range reductions and the exp and sin/cos
# polynomials: 32) and one complex multiply-add (8)
SWEEP_FLOPS_PER_POINT_NODE_DIR = 40.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64 legs")
    ap.add_argument("--no-uniform", action="store_true", help="skip the mixed uniform leg")
    ap.add_argument("--no-near", action="store_true", help="skip the near-interface leg")
    ap.add_argument("--only-near", action="store_true", help="run only the near-interface leg")
    ap.add_argument("--only-batched", action="store_true", help="run only the batched legs")
    ap.add_argument("--only-uniform", action="store_true", help="run only the mixed uniform leg")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB")
    return ap.parse_args()


def recorded_traffic(prefixes, path=TRAFFIC_FILE):
    """HBM bytes per launch of the kernels whose names start with one of
    `prefixes` (averaged over all their dispatches) from a committed counter
    summary, if it was taken on the current kernel sources (else None)."""
    try:
        text = open(path).read()
    except OSError:
        return None
    m = re.search(r"source_sha256:\s*([0-9a-f]+)", text)
    if not m or m.group(1) != source_hash():
        return None
    tot, n = 0.0, 0
    for prefix in prefixes:
        for m in re.finditer(r"^\|\s*%s[^|]*\|\s*(\d+)\s*\|[^\n]*?\|\s*bytes_per_launch=([0-9.eE+]+)" % re.escape(prefix),
                             text, re.M):
            tot += float(m.group(2)) * int(m.group(1))
            n += int(m.group(1))
    return tot / n if n else None


def copy_probe(torch, mib):
    n = mib * (1 << 20) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        torch.mul(a, 1.0, out=b)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe": {"kernel": "elementwise mul by 1 (float32)", "read_bytes": 4 * n,
                                     "write_bytes": 4 * n, "launches": 3}}), flush=True)


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def roofline(st, peak_key, kernel_names, bound="alu", traffic_file=TRAFFIC_FILE):
    """Dominant kernel class of the timed applies against its peak:
    achieved = algorithmic flops per launch / mean launch duration.  The tree
    group (bounding box and tree build, HBM-bound) is reported apart
    (tree_roofline)."""
    nap = max(1, st["timed_applies"])
    cand = {k: v for k, v in st["kernel_ms"].items() if k in kernel_names and st["kernel_launches"][k] > 0}
    dom = max(cand, key=cand.get)
    launches = st["kernel_launches"][dom] / nap
    avg_s = cand[dom] / nap / launches * 1e-3
    flops_launch = st["kernel_flops"][dom] / launches
    achieved = flops_launch / avg_s
    kname = " + ".join(kernel_names[dom])
    traffic = recorded_traffic(kernel_names[dom], traffic_file)
    return {"kernel": kname, "class": dom, "bound": bound, "achieved": achieved / 1e12,
            "peak": PEAK[peak_key] / 1e12, "unit": "TFLOP/s", "frac": achieved / PEAK[peak_key],
            "traffic": traffic, "flops_per_launch": flops_launch, "launches_per_apply": launches,
            "avg_launch_us": avg_s * 1e6, "hbm_GBps_if_traffic": (traffic / avg_s / 1e9) if traffic else None}


# algorithmic HBM bytes of the tree build per point, those of a counting
# sort by leaf (count: coordinates in, leaf key and slot out; scatter: key and
# slot in, index out; leaf order: index and coordinates in, grouped
# coordinates and index out), the yardstick for both grouping forms, plus the
# bounding box (coordinates in) when it is computed, plus each source's
# densities read and written in grouped order
TREE_BYTES_PER_POINT = (16 + 8) + (8 + 4) + (4 + 16 + 16 + 4)
BBOX_BYTES_PER_POINT = 16


def tree_roofline(st, n_points, n_sources, density_bytes, bbox):
    nap = max(1, st["timed_applies"])
    t = st["kernel_ms"]["tree"] / nap * 1e-3
    if t <= 0:
        return None
    by = n_points * (TREE_BYTES_PER_POINT + (BBOX_BYTES_PER_POINT if bbox else 0)) + 2 * n_sources * density_bytes
    return {"kernels": "bounding box and tree build (one group)", "bound": "hbm", "achieved": by / t / 1e9,
            "peak": PEAK["hbm"] / 1e9, "unit": "GB/s", "frac": by / t / PEAK["hbm"], "bytes_per_apply": by,
            "us_per_apply": t * 1e6}


def time_batch(torch, b, items, outs, steps, warmup):
    for _ in range(warmup):
        b.apply(items, outs=outs)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        b.apply(items, outs=outs)
    torch.cuda.synchronize()
    t = (time.perf_counter() - t0) / steps
    # per-class durations: the same merged launches with start/stop events
    b.set_option("timing", "1")
    b.apply(items, outs=outs)
    b.set_option("timing", "reset")
    for _ in range(steps):
        b.apply(items, outs=outs)
    torch.cuda.synchronize()
    st = b.stats()
    b.set_option("timing", "0")
    return t, st


# kernel class -> name prefixes of its merged kernels (every template instance
# and form the plans may choose)
BATCH_KERNELS = {"p2m": ("k_p2m_multi<float", "k_p2m_series_multi<float"),
                 "m2m": ("k_shift_mfma_multi<float, true", "k_up_multi<float"),
                 "m2l": ("k_m2l_mfma_multi<float", "k_m2l_all_multi<float"),
                 "l2l": ("k_shift_mfma_multi<float, false", "k_down_multi<float"),
                 "near_sweep": ("k_near_sweep_multi<float",),
                 "l2p_near": ("k_l2p_multi<float", "k_l2p_near_multi<float")}


def batched_legs(torch, args):
    from paper_1902_08250_amd.lmfmm import Batch, Plan
    inst = workloads.make_batched()
    inter = float(sum(d["src"].shape[1] * d["tgt"].shape[1] * d["q"].shape[0] for d in inst))
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()  # noqa: E731
    items = [(dev(d["src"]), dev(d["q"]), dev(d["tgt"])) for d in inst]
    media = [(d["k"], d["d"]) for d in inst]
    cache = os.path.join(tempfile.mkdtemp(prefix="lmfmm_tune_"), "tune.jsonl")
    t0 = time.perf_counter()
    b = Batch(media, order_set=(12, 16, 20), tol=1e-6, tune_cache=cache)
    outs = b.apply(items)
    torch.cuda.synchronize()
    prep_tuned = time.perf_counter() - t0
    # a second batch over the same instances takes its choices from the cache
    t0 = time.perf_counter()
    b_c = Batch(media, order_set=(12, 16, 20), tol=1e-6, tune_cache=cache)
    outs_c = b_c.apply(items)
    torch.cuda.synchronize()
    prep_cached = time.perf_counter() - t0
    del b_c, outs_c
    t, st = time_batch(torch, b, items, outs, args.steps, args.warmup)
    print(f"[bench] batched mixed: {t * 1e3:.3f} ms/step", file=sys.stderr, flush=True)
    u = [o.cpu().numpy().astype(np.complex128) for o in outs]
    errs = []
    for i in range(len(inst)):
        g = np.load(os.path.join(GOLD, f"oracle_batched_inst{i}.npz"))
        errs.append(rel(u[i][:, g["sel"]], g["u"]))
    out = {"value": inter / t, "ms_per_step": t * 1e3, "interactions_per_step": inter, "stats": st,
           "choices": b.choices(), "prepare_s_tuned": prep_tuned, "prepare_s_from_cache": prep_cached,
           "rel_l2_max_vs_oracle_samples": max(errs), "roofline": roofline(st, "fp32", BATCH_KERNELS),
           "tree_roofline": tree_roofline(st, sum(d["src"].shape[1] + d["tgt"].shape[1] for d in inst),
                                          sum(d["src"].shape[1] for d in inst), 8 * inst[0]["q"].shape[0], False)}
    if not args.no_fp64:
        items64 = [(s, dev(d["q"].astype(np.complex128)), tt) for (s, _, tt), d in zip(items, inst)]
        t0 = time.perf_counter()
        b64 = Batch(media, order_set=(12, 16, 20), tol=1e-10)
        outs64 = b64.apply(items64)
        torch.cuda.synchronize()
        prep64 = time.perf_counter() - t0
        t64, st64 = time_batch(torch, b64, items64, outs64, max(3, args.steps // 2), 1)
        print(f"[bench] batched fp64: {t64 * 1e3:.3f} ms/step", file=sys.stderr, flush=True)
        u64 = [o.cpu().numpy() for o in outs64]
        e64 = []
        for i in range(len(inst)):
            g = np.load(os.path.join(GOLD, f"oracle_batched_inst{i}.npz"))
            e64.append(rel(u64[i][:, g["sel"]], g["u"]))
        out["fp64_batched"] = {"value": inter / t64, "ms_per_step": t64 * 1e3, "tol": 1e-10,
                               "prepare_s_tuned": prep64, "choices": b64.choices(),
                               "rel_l2_max_vs_oracle_samples": max(e64),
                               "kernel_ms_per_apply": {k: v / max(1, st64["timed_applies"])
                                                       for k, v in st64["kernel_ms"].items() if v > 0}}
        out["speedup_mixed_batched_vs_fp64_batched"] = t64 / t
        out["rel_l2_max_mixed_vs_fp64_batched"] = max(rel(a, c) for a, c in zip(u, u64))
        # FP64 plans applied one after another (no batching), for context
        plans = [Plan(d["k"], d["d"], order=16, tol=1e-10) for d in inst]
        os_ = [p.apply(*it) for p, it in zip(plans, items64)]
        torch.cuda.synchronize()
        n64 = max(2, args.steps // 4)
        t0 = time.perf_counter()
        for _ in range(n64):
            for p, it, o in zip(plans, items64, os_):
                p.apply(*it, out=o)
        torch.cuda.synchronize()
        ts = (time.perf_counter() - t0) / n64
        out["fp64_sequential_plans"] = {"value": inter / ts, "ms_per_step": ts * 1e3}
        out["speedup_mixed_batched_vs_fp64_sequential"] = ts / t
    return inst, out


UNIFORM_KERNELS = {"p2m": ("k_p2m<float", "k_p2m_series<float"), "m2m": ("k_shift_mfma<float, true", "k_up<float"),
                   "m2l": ("k_m2l_mfma<float", "k_m2l_all<float"), "l2l": ("k_shift_mfma<float, false", "k_down<float"),
                   "l2p_near": ("k_l2p<float", "k_l2p_near<float")}


def run_plan(torch, Plan, w, precision, steps, warmup, timing=False, domain=None):
    """Times `steps` applies (the second warm-up apply captures the launch
    sequence as a HIP graph, the timed ones replay it).  With timing, the same
    steps are run again kernel by kernel with HIP start/stop events on every
    kernel launch of the apply's stream, for the per-kernel durations.  Also
    returns the time of the plan's first apply, which builds its tables."""
    dt = torch.complex128 if precision == "c128" else torch.complex64
    src = torch.from_numpy(w["src"]).cuda()
    tgt = torch.from_numpy(w["tgt"]).cuda()
    q = torch.from_numpy(w["q"].astype(np.complex128 if precision == "c128" else np.complex64)).cuda()
    u = torch.empty((q.shape[0], tgt.shape[1]), dtype=dt, device="cuda")
    pl = Plan(w["k"], w["d"], order=w["order"], tol=w["tol"] if precision == "c64" else 1e-10, levels=w["levels"])
    if domain:
        pl.set_option("domain", domain)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pl.apply(src, q, tgt, out=u)
    torch.cuda.synchronize()
    cold = time.perf_counter() - t0
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
    return (t1 - t0) / steps, out, st, cold


def uniform_leg(torch, Plan, args):
    w = workloads.make(1)
    inter = float(w["n_src"]) * w["n_tgt"] * w["nrhs"]
    t, u, st, cold = run_plan(torch, Plan, w, "c64", args.steps, args.warmup, timing=True)
    print(f"[bench] uniform mixed: {t * 1e3:.3f} ms/step", file=sys.stderr, flush=True)
    nap = max(1, st["timed_applies"])
    g = np.load(os.path.join(GOLD, "oracle_mixed_uniform_1e5.npz"))
    out = {"workload": w["name"], "n_src": w["n_src"], "n_tgt": w["n_tgt"], "nrhs": w["nrhs"], "order": w["order"],
           "levels": w["levels"], "tol": w["tol"], "dtype": "f32", "value": inter / t, "ms_per_step": t * 1e3,
           "cold_apply_ms": cold * 1e3, "orders_by_level": st["order"],
           "kernel_ms_per_apply": {k: v / nap for k, v in st["kernel_ms"].items() if v > 0},
           "kernel_launches_per_apply": {k: v / nap for k, v in st["kernel_launches"].items() if v > 0},
           "graph_applies_in_timed_region": st["graph_applies"],
           "rel_l2_vs_oracle_samples": rel(u[:, g["sel"]].astype(np.complex128), g["u"]),
           "roofline": roofline(st, "fp32", UNIFORM_KERNELS, traffic_file=UNIFORM_TRAFFIC_FILE),
           "tree_roofline": tree_roofline(st, w["n_src"] + w["n_tgt"], w["n_src"], 8 * w["nrhs"], True)}
    t_dom, u_dom, _, _ = run_plan(torch, Plan, w, "c64", args.steps, args.warmup, domain="0,1,1,-0.95")
    out["fixed_domain"] = {"value": inter / t_dom, "ms_per_step": t_dom * 1e3,
                           "max_abs_diff_vs_auto": float(np.max(np.abs(u_dom - u)))}
    if not args.no_fp64:
        t64, u64, _, cold64 = run_plan(torch, Plan, w, "c128", max(3, args.steps // 4), 1)
        out["fp64"] = {"value": inter / t64, "ms_per_step": t64 * 1e3, "cold_apply_ms": cold64 * 1e3,
                       "rel_l2_vs_oracle_samples": rel(u64[:, g["sel"]], g["u"])}
        out["rel_l2_mixed_vs_fp64"] = rel(u.astype(np.complex128), u64)
    return w, out


def near_leg(torch, Plan, args):
    """The near-interface workload (2e5 sources and targets within 1e-3 of
    the interface, medium k = (40, 60, 50) + 0.01i, d = 0.5, FP64, order 20,
    12 levels): the near field is the x-ordered sweep of the row-0 leaves."""
    w = workloads.make(2)
    inter = float(w["n_src"]) * w["n_tgt"] * w["nrhs"]
    n = max(3, args.steps // 4)
    t, u, st, cold = run_plan(torch, Plan, w, "c128", n, args.warmup, timing=True)
    print(f"[bench] near-interface: {t * 1e3:.3f} ms/step", file=sys.stderr, flush=True)
    nap = max(1, st["timed_applies"])
    sweep_s = st["kernel_ms"]["near_sweep"] / nap * 1e-3
    nodes = st["near_nodes_mid"] + 2 * st["near_nodes_ray"]
    # the plan's count: every point of the row-0 leaves once per direction and
    # node (here all points)
    flops = st["kernel_flops"]["near_sweep"]
    g = np.load(os.path.join(GOLD, "oracle_near_interface_2e5.npz"))
    return {"workload": w["name"], "n_src": w["n_src"], "n_tgt": w["n_tgt"], "order": w["order"],
            "levels": w["levels"], "tol": 1e-10, "dtype": "f64", "steps": n, "value": inter / t,
            "unit": "interactions/s", "ms_per_step": t * 1e3, "cold_apply_ms": cold * 1e3,
            "kernel_ms_per_apply": {k: v / nap for k, v in st["kernel_ms"].items() if v > 0},
            "rel_l2_vs_oracle_samples": rel(u[:, g["sel"]], g["u"]),
            "roofline": {"kernel": "k_near_sweep<double, 1>", "bound": "alu", "achieved": flops / sweep_s / 1e12,
                         "peak": PEAK["fp64"] / 1e12, "unit": "TFLOP/s", "frac": flops / sweep_s / PEAK["fp64"],
                         "traffic": None, "flops_per_launch": flops, "avg_launch_us": sweep_s * 1e6,
                         "nodes": nodes, "flops_per_point_node_direction": SWEEP_FLOPS_PER_POINT_NODE_DIR}}


def cpu_baseline(inst, args):
    """The oracle on this host's cores on a bounded sample of the batched
    workload: seeded targets taken from the instances in turn (one per
    instance per round), each summed over all of its instance's sources and all
    four right-hand sides, until about args.cpu_seconds of CPU work."""
    import oracle
    oracle.build(force=False)
    cores = oracle.max_threads()
    rng = np.random.default_rng(123)
    pairs, t_cpu, done = 0.0, 0.0, 0
    order = rng.permutation(len(inst))
    while t_cpu <= args.cpu_seconds:
        for i in order:
            d = inst[i]
            j = int(rng.integers(d["n"]))
            t0 = time.perf_counter()
            oracle.apply(d["src"], d["q"].astype(np.complex128), d["tgt"][:, j:j + 1], d["k"], d["d"])
            t_cpu += time.perf_counter() - t0
            pairs += float(d["n"]) * d["q"].shape[0]
            done += 1
            if t_cpu > args.cpu_seconds:
                break
    return {"value": pairs / t_cpu, "unit": "interactions/s", "cores": cores, "kind": "oracle",
            "sample": f"{done} seeded targets, one per instance in turn over {len(inst)} instances, "
                      f"x all their sources x 4 rhs ({t_cpu:.1f} s)"}


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
        print(json.dumps({"near_interface": near_leg(torch, Plan, args)}), flush=True)
        return
    if args.only_uniform:
        print(json.dumps({"mixed_uniform_1e5": uniform_leg(torch, Plan, args)[1]}), flush=True)
        return
    print(f"[bench] batched workload: warmup {args.warmup}, steps {args.steps}", file=sys.stderr, flush=True)
    inst, b = batched_legs(torch, args)
    st = b.pop("stats")
    nap = max(1, st["timed_applies"])
    out = {
        "metric": "source-target interactions/s at stated rel-l2 err; mixed+batched vs FP64 FMM",
        "value": b["value"],
        "unit": "interactions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": b["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "batched-16-instances-4rhs-mixed", "instances": len(inst),
                   "n_per_instance": [d["n"] for d in inst], "nrhs": 4, "tol": 1e-6, "order_set": [12, 16, 20],
                   "media": "k1 U[5,30], k2 U[10,60], k3 U[5,40] (+0.01i), d U[0.5,2], seed 3"},
        "roofline": b.pop("roofline"),
        "batched": dict(b, merged_launches_per_apply=st["launches"],
                        kernel_ms_per_apply={k: v / nap for k, v in st["kernel_ms"].items() if v > 0},
                        kernel_launches_per_apply={k: v / nap for k, v in st["kernel_launches"].items() if v > 0}),
    }
    if not args.only_batched:
        if not args.no_uniform:
            _, out["mixed_uniform_1e5"] = uniform_leg(torch, Plan, args)
        if not args.no_near:
            out["near_interface"] = near_leg(torch, Plan, args)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(inst, args)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
