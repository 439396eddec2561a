"""Write the oracle's values at seeded samples of the full-size workloads.

Calls only the oracle and the seeded input generator (no GPU code): each file
holds the sampled indices and the oracle's FP64 direct sums over ALL sources
(or, for the transposed operator, all targets) at those indices.  The GPU
parity tests compare the FMM with these values element by element.

  oracle_mixed_uniform_1e5.npz     100 targets x 1e5 sources
  oracle_near_interface_2e5.npz    100 targets x 2e5 sources
  oracle_backward_1e6_fwd.npz       16 targets x 1e6 sources
  oracle_backward_1e6_adj.npz       16 sources x 1e6 targets (transpose)
  oracle_batched_inst<i>.npz        8 targets per instance x N_i sources, 4 rhs

The densities are those of the workload (complex64 for the mixed workloads)
widened to complex128.  Usage:
  python tests/golden/make_fullsize_goldens.py [--threads N] [name ...]
Existing files are kept unless named explicitly.
"""
import argparse
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from paper_1902_08250_amd import workloads  # noqa: E402

# sample sizes and the seeds of the index draws
SAMPLES = {"mixed_uniform_1e5": (1, 100, 7001), "near_interface_2e5": (2, 100, 7002),
           "backward_1e6_fwd": (4, 16, 7004), "backward_1e6_adj": (4, 16, 7005)}
BATCH_PER_INST, BATCH_SEED = 8, 7003


def sample(n, k, seed):
    return np.sort(np.random.default_rng(seed).choice(n, k, replace=False)).astype(np.int64)


def save(name, **arrs):
    path = os.path.join(HERE, f"oracle_{name}.npz")
    np.savez(path + ".tmp.npz", **arrs)
    os.replace(path + ".tmp.npz", path)
    print("wrote", path, flush=True)


def run_case(name, threads):
    t0 = time.perf_counter()
    if name.startswith("batched_inst"):
        i = int(name[len("batched_inst"):])
        d = workloads.make_batched()[i]
        sel = sample(d["n"], BATCH_PER_INST, BATCH_SEED + 100 * i)
        u = oracle.apply(d["src"], d["q"].astype(np.complex128), d["tgt"][:, sel], d["k"], d["d"],
                         threads=threads)
        save(name, sel=sel, u=u, seed=np.int64(BATCH_SEED + 100 * i))
    else:
        cfg, k, seed = SAMPLES[name]
        w = workloads.make(cfg)
        q = w["q"].astype(np.complex128)
        if name.endswith("_adj"):
            sel = sample(w["n_src"], k, seed)
            wt = w["w"].astype(np.complex128)
            v = oracle.apply_adjoint(w["src"][:, sel], w["tgt"], wt, w["k"], w["d"], threads=threads)
            save(name, sel=sel, v=v, seed=np.int64(seed))
        else:
            sel = sample(w["n_tgt"], k, seed)
            u = oracle.apply(w["src"], q, w["tgt"][:, sel], w["k"], w["d"], threads=threads)
            save(name, sel=sel, u=u, seed=np.int64(seed))
    print(f"{name}: {time.perf_counter() - t0:.0f} s", flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--threads", type=int, default=0)
    ap.add_argument("names", nargs="*")
    a = ap.parse_args()
    oracle.build(force=False)
    allnames = list(SAMPLES) + [f"batched_inst{i}" for i in range(16)]
    names = a.names or [n for n in allnames if not os.path.exists(os.path.join(HERE, f"oracle_{n}.npz"))]
    for n in names:
        run_case(n, a.threads)


if __name__ == "__main__":
    main()
