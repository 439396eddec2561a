"""Mixed-precision uniform workload at full size: N = M = 1e5 in the plain
slabs, medium k = (10, 20, 15) + 0.01i, d = 1, complex64 densities, order 16
on a 7-level quadtree (the benchmark configuration).

  * mixed FMM and FP64 FMM against the oracle at 100 seeded targets, each
    summed over all 1e5 sources (tests/golden/oracle_mixed_uniform_1e5.npz,
    written by make_fullsize_goldens.py): 1e-6 (mixed) and 1e-10 (FP64),
    rel-l2 and worst entry;
  * mixed FMM against the FP64 FMM over all targets (1e-6).
"""
import os
import sys

import numpy as np
import pytest

from paper_1902_08250_amd import workloads
from parity_util import TOL, check

pytestmark = pytest.mark.gpu
GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "oracle_mixed_uniform_1e5.npz")


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def test_mixed_uniform_1e5():
    from paper_1902_08250_amd.lmfmm import Plan
    w = workloads.make(1)
    g = np.load(GOLD)
    sel, ref = g["sel"], g["u"]
    say("mixed-uniform-1e5: mixed FMM and FP64 FMM vs oracle at", sel.size, "targets")
    src, tgt = dev(w["src"]), dev(w["tgt"])
    pl32 = Plan(w["k"], w["d"], order=w["order"], tol=w["tol"], levels=w["levels"])
    u32 = pl32.apply(src, dev(w["q"].astype(np.complex64)), tgt).cpu().numpy().astype(np.complex128)
    pl64 = Plan(w["k"], w["d"], order=w["order"], tol=1e-10, levels=w["levels"])
    u64 = pl64.apply(src, dev(w["q"].astype(np.complex128)), tgt).cpu().numpy()
    say("orders", pl32.stats()["order"], pl64.stats()["order"])
    check(u32[:, sel], ref, TOL["c64"], "mixed vs oracle", say)
    check(u64[:, sel], ref, TOL["c128"], "fp64 vs oracle", say)
    check(u32, u64, TOL["c64"], "mixed vs fp64 fmm (all targets)", say)
