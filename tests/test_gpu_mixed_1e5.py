"""Mixed-precision uniform workload at full size: N = M = 1e5 in the plain
slabs, medium k = (10, 20, 15) + 0.01i, d = 1, complex64 densities, order 16
on a 7-level quadtree (the benchmark configuration).

  * against the FP64 FMM (tol 1e-10) over all targets;
  * against the FP64 GPU direct sum at 1000 seeded targets over all sources;
  * the direct sum against the oracle at 3 of those targets.
"""
import sys

import numpy as np
import pytest

from paper_1902_08250_amd import workloads

pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def test_mixed_uniform_1e5(orc):
    from paper_1902_08250_amd.lmfmm import Plan
    w = workloads.make(1)
    say("mixed-uniform-1e5: mixed FMM, FP64 FMM, direct at 1000 targets")
    src, tgt = dev(w["src"]), dev(w["tgt"])
    pl32 = Plan(w["k"], w["d"], order=w["order"], tol=w["tol"], levels=w["levels"])
    u32 = pl32.apply(src, dev(w["q"].astype(np.complex64)), tgt).cpu().numpy().astype(np.complex128)
    q64 = w["q"].astype(np.complex128)
    pl64 = Plan(w["k"], w["d"], order=w["order"], tol=1e-10, levels=w["levels"])
    u64 = pl64.apply(src, dev(q64), tgt).cpu().numpy()
    rng = np.random.default_rng(1001)
    sel = np.sort(rng.choice(w["n_tgt"], 1000, replace=False))
    d = pl64.direct(src, dev(q64), dev(np.ascontiguousarray(w["tgt"][:, sel]))).cpu().numpy()
    e_mf, e_fd, e_md = rel(u32, u64), rel(u64[:, sel], d), rel(u32[:, sel], d)
    say("rel-l2 mixed vs fp64 fmm", e_mf, "fp64 fmm vs direct", e_fd, "mixed vs direct", e_md,
        "orders", pl32.stats()["order"])
    three = np.array([0, 500, 999])
    ref = orc.apply(w["src"], q64, w["tgt"][:, sel[three]], w["k"], w["d"])
    e_do = rel(d[:, three], ref)
    say("direct vs oracle at 3 targets", e_do)
    assert e_mf < 1e-6 and e_md < 1e-6 and e_fd < 1e-10 and e_do < 1e-12
