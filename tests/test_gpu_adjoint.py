"""Transposed operator and coordinate gradients on the GPU.

  * lmfmm_apply_adjoint against the oracle's transposed direct sum and the
    bilinear identity <w, G q> = <G^T w, q>;
  * lmfmm_grad_coords against the oracle's gradients (derivative integrands)
    and against central differences (h = 1e-5) of the FP64 FMM apply;
  * the mixed-precision gradient against the FP64 one.
"""
import sys

import numpy as np
import pytest

from paper_1902_08250_amd import workloads
from parity_util import TOL, check

pytestmark = pytest.mark.gpu
K, D = workloads.MEDIUM_A


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


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def problem(ns, nt, nrhs, seed):
    rng = np.random.default_rng(seed)
    return workloads.draw_instance(rng, ns, nt, (0, 1), (0.05, 1), (-0.95, -0.05), nrhs)


@pytest.fixture(scope="module")
def cuda():
    import torch
    assert torch.cuda.is_available()
    return torch


@pytest.mark.parametrize("levels", [1, 3])
def test_adjoint_vs_oracle(cuda, orc, levels):
    from paper_1902_08250_amd.lmfmm import Plan
    say("adjoint 300x200 vs oracle, levels", levels)
    src, tgt, q, w = problem(300, 200, 2, 21)
    ref = orc.apply_adjoint(src, tgt, w, K, D)
    pl = Plan(K, D, order=20, tol=1e-10, levels=levels)
    v = host(pl.apply_adjoint(dev(src), dev(tgt), dev(w)))
    err = rel(v, ref)
    say("adjoint rel-l2", err)
    assert err < 1e-10


def test_adjoint_bilinear_identity(cuda):
    from paper_1902_08250_amd.lmfmm import Plan
    say("adjoint bilinear identity 20000x15000")
    src, tgt, q, w = problem(20000, 15000, 3, 22)
    pl = Plan(K, D, order=20, tol=1e-10, levels=5)
    u = host(pl.apply(dev(src), dev(q), dev(tgt)))
    v = host(pl.apply_adjoint(dev(src), dev(tgt), dev(w)))
    for r in range(3):
        lhs = np.sum(w[r] * u[r])
        rhs = np.sum(v[r] * q[r])
        say("identity", r, abs(lhs - rhs) / abs(lhs))
        assert abs(lhs - rhs) < 1e-10 * abs(lhs)


def test_adjoint_mixed(cuda):
    from paper_1902_08250_amd.lmfmm import Plan
    say("adjoint mixed vs fp64 20000x15000")
    src, tgt, q, w = problem(20000, 15000, 1, 23)
    pl = Plan(K, D, order=16, tol=1e-6, levels=5)
    v64 = host(pl.apply_adjoint(dev(src), dev(tgt), dev(w)))
    v32 = host(pl.apply_adjoint(dev(src), dev(tgt), dev(w.astype(np.complex64))))
    check(v32, v64, TOL["c64"], "mixed adjoint vs fp64", say)


@pytest.mark.parametrize("levels", [1, 3])
def test_grad_vs_oracle(cuda, orc, levels):
    from paper_1902_08250_amd.lmfmm import Plan
    say("grad 150x120 vs oracle, levels", levels)
    src, tgt, q, w = problem(150, 120, 2, 24)
    rs, rt = orc.grad_coords(src, q, tgt, w, K, D)
    pl = Plan(K, D, order=20, tol=1e-10, levels=levels)
    ds, dt = pl.grad_coords(dev(src), dev(q), dev(tgt), dev(w))
    ds, dt = host(ds), host(dt)
    es, et = rel(ds, rs), rel(dt, rt)
    say("grad rel-l2 src", es, "tgt", et)
    assert es < 1e-9 and et < 1e-9


def test_grad_central_differences(cuda):
    from paper_1902_08250_amd.lmfmm import Plan
    say("grad vs central differences 6000x5000")
    src, tgt, q, w = problem(6000, 5000, 1, 25)
    pl = Plan(K, D, order=20, tol=1e-10, levels=4)
    ds, dt = pl.grad_coords(dev(src), dev(q), dev(tgt), dev(w))
    ds, dt = host(ds), host(dt)

    def L(s, t):
        return float(np.real(np.sum(w * host(pl.apply(dev(s), dev(q), dev(t))))))

    h = 1e-5
    rng = np.random.default_rng(5)
    for which in ("s", "t"):
        arr, grad = (src, ds) if which == "s" else (tgt, dt)
        for idx in rng.choice(arr.shape[1], 3, replace=False):
            for comp in (0, 1):
                p_, m_ = arr.copy(), arr.copy()
                p_[comp, idx] += h
                m_[comp, idx] -= h
                fd = (L(p_, tgt) - L(m_, tgt)) / (2 * h) if which == "s" else (L(src, p_) - L(src, m_)) / (2 * h)
                say("fd", which, comp, idx, fd, grad[comp, idx])
                assert abs(fd - grad[comp, idx]) < 1e-5 * max(1.0, abs(grad[comp, idx]))


def test_grad_mixed_vs_fp64(cuda):
    from paper_1902_08250_amd.lmfmm import Plan
    say("grad mixed vs fp64 20000x15000")
    src, tgt, q, w = problem(20000, 15000, 1, 26)
    pl = Plan(K, D, order=16, tol=1e-6, levels=5)
    ds64, dt64 = pl.grad_coords(dev(src), dev(q), dev(tgt), dev(w))
    ds32, dt32 = pl.grad_coords(dev(src), dev(q.astype(np.complex64)), dev(tgt), dev(w.astype(np.complex64)))
    check(host(ds32), host(ds64), TOL["c64"], "mixed source gradient vs fp64", say)
    check(host(dt32), host(dt64), TOL["c64"], "mixed target gradient vs fp64", say)


def test_autograd_function(cuda):
    import torch
    from paper_1902_08250_amd.autograd import lmfmm_apply
    from paper_1902_08250_amd.lmfmm import Plan
    say("autograd function 3000x2500")
    src, tgt, q, w = problem(3000, 2500, 2, 27)
    pl = Plan(K, D, order=20, tol=1e-10, levels=4)
    s = dev(src).requires_grad_(True)
    t = dev(tgt).requires_grad_(True)
    qq = dev(q).requires_grad_(True)
    ww = dev(w)
    u = lmfmm_apply(pl, s, qq, t)
    L = (ww * u).sum().real
    L.backward()
    v = host(pl.apply_adjoint(dev(src), dev(tgt), dev(w)))
    ds, dt = pl.grad_coords(dev(src), dev(q), dev(tgt), dev(w))
    assert rel(host(qq.grad), np.conj(v)) < 1e-13
    assert rel(host(s.grad), host(ds)) < 1e-13
    assert rel(host(t.grad), host(dt)) < 1e-13
