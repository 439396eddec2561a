"""Parity of the HIP path with the FP64 oracle (GPU).

Every case prints its name before touching the GPU.  The 512 x 512 plain
workload is compared with the oracle's stored result
(tests/golden/oracle_plain512_u.npy, written by make_oracle_golden.py);
smaller cases call the oracle directly.
"""
import os
import sys

import numpy as np
import pytest

from paper_1902_08250_amd import workloads

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))


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


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


@pytest.fixture(scope="module")
def plain():
    return workloads.make(0)


@pytest.fixture(scope="module")
def golden512():
    path = os.path.join(HERE, "golden", "oracle_plain512_u.npy")
    return np.load(path)


def test_direct_matches_oracle(torch_cuda, plain, orc):
    from paper_1902_08250_amd.lmfmm import Plan
    say("direct 128x96 vs oracle")
    src, tgt, q = plain["src"][:, :128], plain["tgt"][:, :96], plain["q"][:, :128]
    ref = orc.apply(src, q, tgt, plain["k"], plain["d"])
    pl = Plan(plain["k"], plain["d"], order=20, tol=1e-10)
    u = host(pl.direct(dev(src), dev(q), dev(tgt)))
    err = rel(u, ref)
    say("direct rel-l2", err)
    assert err < 1e-12


def test_fmm_plain512_vs_oracle(torch_cuda, plain, golden512):
    from paper_1902_08250_amd.lmfmm import Plan
    say("fmm 512x512 L=3 tol=1e-10 vs oracle")
    pl = Plan(plain["k"], plain["d"], order=20, tol=1e-10, levels=3)
    u = host(pl.apply(dev(plain["src"]), dev(plain["q"]), dev(plain["tgt"])))
    err = rel(u, golden512)
    say("fmm rel-l2", err, pl.stats()["order"])
    assert err < 1e-10


def test_fmm_plain512_fixed_order20(torch_cuda, plain, golden512):
    """The workload's nominal order p = 20 at every level (error reported)."""
    from paper_1902_08250_amd.lmfmm import Plan
    say("fmm 512x512 L=3 fixed p=20")
    pl = Plan(plain["k"], plain["d"], order=20, tol=1e-10, levels=3, fixed_order=True)
    u = host(pl.apply(dev(plain["src"]), dev(plain["q"]), dev(plain["tgt"])))
    err = rel(u, golden512)
    say("fmm p=20 rel-l2", err)
    assert err < 1e-6


@pytest.mark.parametrize("levels", [1, 2, 4, 5])
def test_fmm_levels_vs_oracle(torch_cuda, plain, golden512, levels):
    from paper_1902_08250_amd.lmfmm import Plan
    say("fmm 512x512 levels", levels)
    pl = Plan(plain["k"], plain["d"], order=20, tol=1e-10, levels=levels)
    u = host(pl.apply(dev(plain["src"]), dev(plain["q"]), dev(plain["tgt"])))
    err = rel(u, golden512)
    say("rel-l2", err)
    assert err < 1e-10


def test_mixed_plain512_vs_oracle(torch_cuda, plain, golden512):
    from paper_1902_08250_amd.lmfmm import Plan
    say("mixed 512x512 L=3 tol=1e-6")
    pl = Plan(plain["k"], plain["d"], order=16, tol=1e-6, levels=3)
    q32 = plain["q"].astype(np.complex64)
    u = host(pl.apply(dev(plain["src"]), dev(q32), dev(plain["tgt"])))
    err = rel(u.astype(np.complex128), golden512)
    say("mixed rel-l2", err)
    assert err < 1e-5
