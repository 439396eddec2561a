"""The other field components on the GPU (Section 3): g_2^b (middle layer,
from the bottom interface, targets imaged to y' = -y - 2d), g_1^s (top layer,
y' = -y), g_3^s (bottom layer) of the three-layer medium k = (10, 20, 15) +
0.01i, d = 1, and the impedance half-space (Example 3; k = 10 + 0.01i,
alpha = 1; targets above the interface, y' = -y).  Each is compared with the
oracle of the same component: the FP64 FMM at 1e-10 and the mixed FMM at
1e-6 (rel-l2 and worst entry), the transposed operator at 1e-10, the GPU
direct sum at 1e-12, the coordinate gradients at 1e-9; and cases with every
point within 1e-3 of the interface for the components whose image targets
come close to the sources (g_1^s and the impedance half-space), so that the
near-field sweep runs on imaged targets."""
import sys

import numpy as np
import pytest

from paper_1902_08250_amd import workloads
from parity_util import TOL, check

pytestmark = pytest.mark.gpu
K3 = workloads.MEDIUM_A[0]
D = 1.0
KI = (10 + 0.01j, 10 + 0.01j, 10 + 0.01j)
ALPHA = 1.0
# component -> (medium, target y range)
CASES = {"2b": (K3, (-0.95, -0.05)), "1s": (K3, (0.05, 1.0)), "3s": (K3, (-1.95, -1.05)),
         "impedance": (KI, (0.05, 1.0))}
ORC = {"2b": "2b", "1s": "1s", "3s": "3s", "impedance": "imp"}


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy()


def problem(comp, ns, nt, nrhs, seed, near=False):
    rng = np.random.default_rng(seed)
    yt = CASES[comp][1]
    ys = (0.05, 1.0)
    if near:
        ys, yt = (1e-4, 1e-3), (1e-4, 1e-3)
    return workloads.draw_instance(rng, ns, nt, (0, 1), ys, yt, nrhs)


def plan(comp, tol, order, levels=None):
    from paper_1902_08250_amd.lmfmm import Plan
    k = CASES[comp][0]
    return Plan(k, D, order=order, tol=tol, levels=levels, component=comp,
                alpha=ALPHA if comp == "impedance" else None)


def oracle_kw(comp):
    return dict(comp=ORC[comp], alpha=ALPHA if comp == "impedance" else 0.0)


@pytest.mark.parametrize("comp", list(CASES))
def test_component_apply(comp, orc):
    say("component", comp, ": FMM (FP64, mixed) and direct vs oracle, 3000 x 2000, 2 rhs")
    k = CASES[comp][0]
    src, tgt, q, _ = problem(comp, 3000, 2000, 2, 61)
    sel = np.arange(0, 2000, 40)
    ref = orc.apply(src, q, tgt[:, sel], k, D, **oracle_kw(comp))
    pl = plan(comp, 1e-10, 20)
    u = host(pl.apply(dev(src), dev(q), dev(tgt)))
    say("levels", pl.stats()["levels"], "orders", pl.stats()["order"])
    check(u[:, sel], ref, TOL["c128"], f"{comp} fp64 fmm vs oracle", say)
    d = host(pl.direct(dev(src), dev(q), dev(np.ascontiguousarray(tgt[:, sel]))))
    check(d, ref, 1e-12, f"{comp} gpu direct vs oracle", say)
    pl32 = plan(comp, 1e-6, 16)
    u32 = host(pl32.apply(dev(src), dev(q.astype(np.complex64)), dev(tgt)))
    check(u32[:, sel], ref, TOL["c64"], f"{comp} mixed fmm vs oracle", say)


@pytest.mark.parametrize("comp", ["1s", "impedance"])
def test_component_near_interface(comp, orc):
    say("component", comp, ": every point within 1e-3 of the interface, 20000 x 20000")
    k = CASES[comp][0]
    src, tgt, q, _ = problem(comp, 20000, 20000, 1, 62, near=True)
    sel = np.linspace(0, 19999, 8).astype(int)
    ref = orc.apply(src, q, tgt[:, sel], k, D, **oracle_kw(comp))
    pl = plan(comp, 1e-10, 20, levels=9)
    u = host(pl.apply(dev(src), dev(q), dev(tgt)))
    check(u[:, sel], ref, TOL["c128"], f"{comp} near interface fp64 vs oracle", say)


@pytest.mark.parametrize("comp", list(CASES))
def test_component_adjoint_and_gradients(comp, orc):
    say("component", comp, ": transposed operator and gradients vs oracle")
    k = CASES[comp][0]
    src, tgt, q, w = problem(comp, 300, 200, 2, 63)
    pl = plan(comp, 1e-10, 20, levels=3)
    v = host(pl.apply_adjoint(dev(src), dev(tgt), dev(w)))
    rv = orc.apply_adjoint(src, tgt, w, k, D, **oracle_kw(comp))
    check(v, rv, TOL["c128"], f"{comp} transposed vs oracle", say)
    ds, dt = pl.grad_coords(dev(src), dev(q), dev(tgt), dev(w))
    rs, rt = orc.grad_coords(src, q, tgt, w, k, D, **oracle_kw(comp))
    check(host(ds), rs, 1e-9, f"{comp} source gradient vs oracle", say)
    check(host(dt), rt, 1e-9, f"{comp} target gradient vs oracle", say)
