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
from parity_util import TOL, check

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
    say("orders", pl.stats()["order"])
    check(u, golden512, TOL["c128"], "fmm 512x512 vs oracle", say)


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
    say("mixed", pl.stats()["order"])
    check(u, golden512, TOL["c64"], "mixed 512x512 vs oracle", say)


@pytest.fixture(scope="module")
def mid():
    """4000 x 3000 points in the plain workload's slabs, 11 right-hand sides."""
    rng = np.random.default_rng(77)
    src, tgt, q, w = workloads.draw_instance(rng, 4000, 3000, (0, 1), (0.05, 1), (-0.95, -0.05), 11)
    return dict(src=src, tgt=tgt, q=q, w=w, k=workloads.MEDIUM_A[0], d=workloads.MEDIUM_A[1])


@pytest.fixture(scope="module")
def mid_direct(torch_cuda, mid):
    from paper_1902_08250_amd.lmfmm import Plan
    say("direct 4000x3000 nrhs=11")
    pl = Plan(mid["k"], mid["d"], order=20, tol=1e-10)
    return host(pl.direct(dev(mid["src"]), dev(mid["q"]), dev(mid["tgt"])))


def test_mid_direct_sample_vs_oracle(mid, mid_direct, orc):
    say("direct 4000x3000 sampled rows vs oracle")
    sel = np.arange(0, 3000, 150)
    ref = orc.apply(mid["src"], mid["q"][:2], mid["tgt"][:, sel], mid["k"], mid["d"])
    assert rel(mid_direct[:2, sel], ref) < 1e-12


@pytest.mark.parametrize("levels", [3, 4, 5, 6])
def test_mid_fmm_vs_direct(torch_cuda, mid, mid_direct, levels):
    from paper_1902_08250_amd.lmfmm import Plan
    say("fmm 4000x3000 nrhs=11 levels", levels)
    pl = Plan(mid["k"], mid["d"], order=20, tol=1e-10, levels=levels)
    u = host(pl.apply(dev(mid["src"]), dev(mid["q"]), dev(mid["tgt"])))
    err = rel(u, mid_direct)
    say("rel-l2", err, pl.stats()["order"])
    assert err < 1e-10
    # every right-hand side individually
    for r in range(u.shape[0]):
        assert rel(u[r], mid_direct[r]) < 1e-10


@pytest.mark.parametrize("levels", [2, 4, 7])
def test_p2m_forms_match_direct(torch_cuda, mid, mid_direct, levels):
    """P2M by the ascending series (default where k1 R allows it) and by the
    recurrence form (option p2m_series = 0), FP64 and mixed, 11 right-hand
    sides (three chunks of four), against the GPU direct sum.  Level 2 puts
    hundreds of points in a leaf (64 lanes per leaf in the series form), level
    7 about one."""
    from paper_1902_08250_amd.lmfmm import Plan
    say("P2M series / recurrence, 4000x3000 nrhs=11 levels", levels)
    for prec, tol in (("c128", 1e-10), ("c64", TOL["c64"])):
        q = mid["q"] if prec == "c128" else mid["q"].astype(np.complex64)
        for ser in ("1", "0"):
            pl = Plan(mid["k"], mid["d"], order=20 if prec == "c128" else 16, tol=1e-10 if prec == "c128" else 1e-6,
                      levels=levels)
            pl.set_option("p2m_series", ser)
            u = host(pl.apply(dev(mid["src"]), dev(q), dev(mid["tgt"])))
            check(u, mid_direct, tol, f"{prec} L={levels} p2m_series={ser} vs direct", say)


def test_p2m_large_k1r_uses_recurrence_form(torch_cuda):
    """A top layer with k1 = 60: at three levels the leaves' k1 R is about
    5.3, beyond the series form, so P2M takes the recurrence form whatever the
    option says; FP64 and mixed FMM against the GPU direct sum."""
    from paper_1902_08250_amd.lmfmm import Plan
    rng = np.random.default_rng(78)
    src, tgt, q, _ = workloads.draw_instance(rng, 3000, 2000, (0, 1), (0.05, 1), (-0.95, -0.05), 2)
    k = (60 + 0.01j, 40 + 0.01j, 30 + 0.01j)
    say("k1 = 60, 3000x2000, levels 3")
    ref = host(Plan(k, 1.0, order=20, tol=1e-10).direct(dev(src), dev(q), dev(tgt)))
    for prec, tol in (("c128", 1e-10), ("c64", TOL["c64"])):
        qq = q if prec == "c128" else q.astype(np.complex64)
        pl = Plan(k, 1.0, order=20 if prec == "c128" else 16, tol=1e-10 if prec == "c128" else 1e-6, levels=3)
        u = host(pl.apply(dev(src), dev(qq), dev(tgt)))
        say("orders", pl.stats()["order"])
        check(u, ref, tol, f"{prec} k1=60 L=3 vs direct", say)


@pytest.mark.parametrize("nrhs", [1, 2, 3, 5])
def test_rhs_counts_and_forms_match_direct(torch_cuda, nrhs):
    """1, 2, 3 and 5 right-hand sides (densities padded to 1, 2, 4 and 2 x 4 in
    the recurrence-form P2M; the M2L form chosen by their number: vector below
    4 in FP32 and 3 in FP64), with M2L forced to either form and P2M in either
    form, FP64 and mixed, 2500 x 2000 at 5 levels (about 3 sources per leaf),
    against the GPU direct sum."""
    from paper_1902_08250_amd.lmfmm import Plan
    rng = np.random.default_rng(90 + nrhs)
    src, tgt, q, _ = workloads.draw_instance(rng, 2500, 2000, (0, 1), (0.05, 1), (-0.95, -0.05), nrhs)
    k, d = workloads.MEDIUM_A
    ref = host(Plan(k, d, order=20, tol=1e-10).direct(dev(src), dev(q), dev(tgt)))
    say("nrhs", nrhs, "2500x2000 levels 5: m2l auto/1/0 x p2m series/recurrence")
    for prec, tol in (("c128", 1e-10), ("c64", TOL["c64"])):
        qq = q if prec == "c128" else q.astype(np.complex64)
        for m2l, ser in (("auto", "1"), ("1", "0"), ("0", "0"), ("auto", "0")):
            pl = Plan(k, d, order=20 if prec == "c128" else 16, tol=1e-10 if prec == "c128" else 1e-6, levels=5)
            pl.set_option("m2l_mfma", m2l)
            pl.set_option("p2m_series", ser)
            u = host(pl.apply(dev(src), dev(qq), dev(tgt)))
            check(u, ref, tol, f"{prec} nrhs={nrhs} m2l_mfma={m2l} p2m_series={ser} vs direct", say)


@pytest.mark.parametrize("levels", [2, 5, 7])
def test_eval_levels_match_leaf_evaluation(torch_cuda, mid, mid_direct, levels):
    """Leaves evaluating the expansion of the level where their far field is
    complete (default) against every leaf evaluating its own shifted expansion
    (option eval_levels = 0), with M2M and L2L on the matrix cores (default)
    and on the vector units (shift_mfma = 0), FP64 and mixed, 11 right-hand
    sides; each against the GPU direct sum."""
    from paper_1902_08250_amd.lmfmm import Plan
    say("eval levels on/off, shifts on matrix cores/vector units, 4000x3000 nrhs=11 levels", levels)
    for prec, tol in (("c128", 1e-10), ("c64", TOL["c64"])):
        q = mid["q"] if prec == "c128" else mid["q"].astype(np.complex64)
        for ev, sm in (("1", "1"), ("0", "1"), ("1", "0"), ("0", "0")):
            pl = Plan(mid["k"], mid["d"], order=20 if prec == "c128" else 16, tol=1e-10 if prec == "c128" else 1e-6,
                      levels=levels)
            pl.set_option("eval_levels", ev)
            pl.set_option("shift_mfma", sm)
            u = host(pl.apply(dev(mid["src"]), dev(q), dev(mid["tgt"])))
            check(u, mid_direct, tol, f"{prec} L={levels} eval_levels={ev} shift_mfma={sm} vs direct", say)


def test_mid_mixed_vs_fp64(torch_cuda, mid, mid_direct):
    from paper_1902_08250_amd.lmfmm import Plan
    say("mixed 4000x3000 nrhs=11 levels 5")
    pl = Plan(mid["k"], mid["d"], order=16, tol=1e-6, levels=5)
    u = host(pl.apply(dev(mid["src"]), dev(mid["q"].astype(np.complex64)), dev(mid["tgt"])))
    check(u, mid_direct, TOL["c64"], "mixed 4000x3000 nrhs=11 vs direct", say)


@pytest.mark.parametrize("levels", [2, 5, 8, 9])
def test_tree_sort_forms(torch_cuda, mid, mid_direct, levels):
    """Both groupings of the points by leaf, the radix sort and the counting
    sort (option tree_sort), list every leaf's points in increasing original
    index, so the results agree bit for bit.  Level 2 has 12 leaves (one
    4-bit digit pass of the radix sort), level 5 about 540 (two passes);
    levels 8 and 9 have about 3e4 and 1.3e5 leaves for 7000 points (15- and
    17-bit keys: two and three passes), so most leaf ranges are empty runs
    between occupied leaves.  FP64 against the GPU direct sum."""
    from paper_1902_08250_amd.lmfmm import Plan
    out = {}
    for form in ("radix", "count"):
        say("tree_sort", form, "4000x3000 nrhs=11 levels", levels)
        pl = Plan(mid["k"], mid["d"], order=20, tol=1e-10, levels=levels)
        pl.set_option("tree_sort", form)
        out[form] = host(pl.apply(dev(mid["src"]), dev(mid["q"]), dev(mid["tgt"])))
        check(out[form], mid_direct, 1e-10, f"c128 L={levels} tree_sort={form} vs direct", say)
    assert np.array_equal(out["radix"], out["count"])
    from paper_1902_08250_amd.lmfmm import LMFMMError
    with pytest.raises(LMFMMError, match="tree_sort"):
        pl.set_option("tree_sort", "bucket")


def test_deterministic(torch_cuda, mid):
    from paper_1902_08250_amd.lmfmm import Plan
    say("determinism 4000x3000")
    pl = Plan(mid["k"], mid["d"], order=20, tol=1e-10, levels=5)
    a = host(pl.apply(dev(mid["src"]), dev(mid["q"]), dev(mid["tgt"])))
    b = host(pl.apply(dev(mid["src"]), dev(mid["q"]), dev(mid["tgt"])))
    assert np.array_equal(a, b)


def test_edge_cases(torch_cuda, plain, orc):
    import torch
    from paper_1902_08250_amd.lmfmm import Plan, LMFMMError
    say("edge cases")
    pl = Plan(plain["k"], plain["d"], order=20, tol=1e-10)
    src, tgt, q = dev(plain["src"]), dev(plain["tgt"]), dev(plain["q"])
    # no targets
    u = pl.apply(src, q, tgt[:, :0].contiguous())
    assert u.shape == (1, 0)
    # no sources: zero field
    u = host(pl.apply(src[:, :0].contiguous(), q[:, :0].contiguous(), tgt))
    assert np.all(u == 0)
    # one source, one target
    s1, t1, q1 = plain["src"][:, :1], plain["tgt"][:, :1], plain["q"][:, :1]
    u = host(pl.apply(dev(s1), dev(q1), dev(t1)))
    ref = orc.apply(s1, q1, t1, plain["k"], plain["d"])
    assert rel(u, ref) < 1e-12
    # all points in a tiny cluster (one leaf) near the interface
    rng = np.random.default_rng(3)
    sc = np.stack([0.5 + 1e-3 * rng.random(50), 1e-4 + 1e-3 * rng.random(50)])
    tc = np.stack([0.5 + 1e-3 * rng.random(40), -1e-4 - 1e-3 * rng.random(40)])
    qc = (rng.standard_normal((1, 50)) + 1j * rng.standard_normal((1, 50)))
    u = host(pl.apply(dev(sc), dev(qc), dev(tc)))
    ref = orc.apply(sc, qc, tc, plain["k"], plain["d"])
    assert rel(u, ref) < 1e-10
    # a point in the wrong layer is rejected
    bad = plain["tgt"].copy()
    bad[1, 5] = 0.2
    with pytest.raises(LMFMMError):
        pl.apply(src, q, dev(bad))
    # the largest number of right-hand sides (64), FP64 and mixed, against the
    # direct sum (itself checked against the oracle)
    q64 = rng.standard_normal((64, 512)) + 1j * rng.standard_normal((64, 512))
    ref = host(pl.direct(src, dev(q64), tgt))
    u = host(pl.apply(src, dev(q64), tgt))
    say("64 rhs rel-l2", rel(u, ref))
    assert rel(u, ref) < 1e-10
    pl32 = Plan(plain["k"], plain["d"], order=16, tol=1e-6)
    u32 = host(pl32.apply(src, dev(q64.astype(np.complex64)), tgt))
    check(u32, ref, TOL["c64"], "64 rhs mixed vs direct", say)


def test_table_cache_follows_row_counts(torch_cuda, plain, orc):
    """Two applies on one plan with the same root width and levels but point
    sets of different depth: the second must match a fresh plan (the class
    sets of the interface rows and of the coarsest level differ)."""
    from paper_1902_08250_amd.lmfmm import Plan
    say("table cache: shallow then deep point sets, same root width")
    rng = np.random.default_rng(11)
    k, d = plain["k"], plain["d"]
    s1, t1, q1, _ = workloads.draw_instance(rng, 3000, 2000, (0, 1), (0.05, 0.1), (-0.1, -0.05), 1)
    s2, t2, q2, _ = workloads.draw_instance(rng, 3000, 2000, (0, 1), (0.05, 0.45), (-0.45, -0.05), 1)
    pl = Plan(k, d, order=20, tol=1e-10, levels=4)
    pl.apply(dev(s1), dev(q1), dev(t1))
    u_reused = host(pl.apply(dev(s2), dev(q2), dev(t2)))
    u_fresh = host(Plan(k, d, order=20, tol=1e-10, levels=4).apply(dev(s2), dev(q2), dev(t2)))
    assert np.array_equal(u_reused, u_fresh)
    sel = np.arange(0, 2000, 100)
    ref = orc.apply(s2, q2, t2[:, sel], k, d)
    err = rel(u_reused[:, sel], ref)
    say("rel-l2 vs oracle", err)
    assert err < 1e-10


@pytest.mark.parametrize("precision", ["c128", "c64"])
def test_graph_replay_matches_direct(torch_cuda, mid, precision):
    """Repeated applies on fixed buffers: the first launches kernel by kernel,
    the second captures a HIP graph, later ones replay it.  The densities are
    rewritten in place between applies (eager work and a synchronisation in
    between); every replay must equal the kernel-by-kernel result bit for bit."""
    import torch
    from paper_1902_08250_amd.lmfmm import Plan
    say("graph replay vs direct launches", precision)
    dt = np.complex128 if precision == "c128" else np.complex64
    tol = 1e-10 if precision == "c128" else 1e-6
    pl = Plan(mid["k"], mid["d"], order=16, tol=tol, levels=5)
    ref_pl = Plan(mid["k"], mid["d"], order=16, tol=tol, levels=5)
    ref_pl.set_option("graph", "0")
    src, tgt = dev(mid["src"]), dev(mid["tgt"])
    q = dev(mid["q"][:3].astype(dt))
    u = torch.empty((3, tgt.shape[1]), dtype=q.dtype, device="cuda")
    rng = np.random.default_rng(8)
    for it in range(7):
        if it == 5:  # timing mode launches kernel by kernel with per-kernel events
            pl.set_option("timing", "1")
        new = rng.standard_normal((3, src.shape[1])) + 1j * rng.standard_normal((3, src.shape[1]))
        q.copy_(torch.from_numpy(new.astype(dt)).cuda())
        torch.cuda.synchronize()
        pl.apply(src, q, tgt, out=u)
        got = host(u)
        want = host(ref_pl.apply(src, q, tgt))
        assert np.array_equal(got, want), f"apply {it}"
    st = pl.stats()
    say("timed applies", st["timed_applies"], "graph applies", st["graph_applies"], "k_down ms",
        st["kernel_ms"]["m2l"])
    assert st["kernel_ms"]["m2l"] > 0
    assert st["graph_applies"] == 4 and st["timed_applies"] == 2


def test_large_leaves(torch_cuda, plain):
    """Leaves of about 6000 and 300 points (the per-leaf ordering runs in the
    scratch array and in LDS; a block's points take several chunks) next to
    small ones, for sources and for targets: FMM against the direct sum, and two
    applies bit for bit equal."""
    from paper_1902_08250_amd.lmfmm import Plan
    say("large leaves: clusters of 6000 and 300 sources and of 3000 and 700 targets, levels 3")
    rng = np.random.default_rng(21)
    k, d = plain["k"], plain["d"]
    sa = np.stack([0.2 + 5e-4 * rng.random(6000), 0.3 + 5e-4 * rng.random(6000)])
    sb = np.stack([0.7 + 1e-3 * rng.random(300), 0.6 + 1e-3 * rng.random(300)])
    su = np.stack([rng.random(500), 0.05 + 0.95 * rng.random(500)])
    src = np.ascontiguousarray(np.concatenate([sa, sb, su], axis=1)[:, rng.permutation(6800)])
    ta = np.stack([0.4 + 5e-4 * rng.random(3000), -0.5 - 5e-4 * rng.random(3000)])
    tb = np.stack([0.9 + 1e-3 * rng.random(700), -0.2 - 1e-3 * rng.random(700)])
    tu = np.stack([rng.random(400), -0.05 - 0.9 * rng.random(400)])
    tgt = np.ascontiguousarray(np.concatenate([ta, tb, tu], axis=1)[:, rng.permutation(4100)])
    q = rng.standard_normal((2, 6800)) + 1j * rng.standard_normal((2, 6800))
    pl = Plan(k, d, order=20, tol=1e-10, levels=3)
    pl.set_option("graph", "0")
    u1 = host(pl.apply(dev(src), dev(q), dev(tgt)))
    u2 = host(pl.apply(dev(src), dev(q), dev(tgt)))
    assert np.array_equal(u1, u2)
    ref = host(pl.direct(dev(src), dev(q), dev(tgt)))
    err = rel(u1, ref)
    say("rel-l2 vs direct", err)
    assert err < 1e-10
    # one right-hand side in mixed precision (the kernels without per-rhs loops)
    pl32 = Plan(k, d, order=16, tol=1e-6, levels=3)
    u32 = host(pl32.apply(dev(src), dev(q[:1].astype(np.complex64)), dev(tgt)))
    check(u32, ref[:1], TOL["c64"], "large leaves, mixed, one rhs vs direct", say)


def test_fixed_domain(torch_cuda, mid, mid_direct):
    """With the domain given up front there is no bounding-box readback: the
    result matches the direct sum, and a point outside the domain is reported
    by the device-side check through sync_status."""
    from paper_1902_08250_amd.lmfmm import Plan, LMFMMError
    say("fixed domain 4000x3000 nrhs=11, levels 5")
    pl = Plan(mid["k"], mid["d"], order=20, tol=1e-10, levels=5)
    pl.set_option("domain", "0,1,1,-0.95")
    u = host(pl.apply(dev(mid["src"]), dev(mid["q"]), dev(mid["tgt"])))
    pl.sync_status()
    err = rel(u, mid_direct)
    say("rel-l2 vs direct", err)
    assert err < 1e-10
    bad = mid["src"].copy()
    bad[0, 7] = 1.5  # x outside [0, 1]
    pl.apply(dev(bad), dev(mid["q"]), dev(mid["tgt"]))
    with pytest.raises(LMFMMError):
        pl.sync_status()
    # the next apply with valid points clears the flag
    pl.apply(dev(mid["src"]), dev(mid["q"]), dev(mid["tgt"]))
    pl.sync_status()


def test_error_decays_with_order(torch_cuda, plain, golden512):
    """Truncation error of the expansions (Theorem 1 and the translation
    lemmas of Section 3): at a fixed order p at every level, the error
    against the oracle falls geometrically in p until it reaches the FP64
    rounding floor."""
    from paper_1902_08250_amd.lmfmm import Plan
    errs = []
    for p in (12, 16, 20, 24, 28, 32):
        say("fmm 512x512 L=3 fixed p =", p)
        pl = Plan(plain["k"], plain["d"], order=p, tol=1e-10, levels=3, fixed_order=True)
        u = host(pl.apply(dev(plain["src"]), dev(plain["q"]), dev(plain["tgt"])))
        errs.append(rel(u, golden512))
    say("rel-l2 by order", errs)
    for a, b in zip(errs, errs[1:]):
        if a > 1e-10:
            assert b < 0.6 * a
    assert errs[-1] < 1e-9


@pytest.mark.parametrize("precision", ["c128", "c64"])
def test_speculative_replay_follows_moving_points(torch_cuda, mid, precision):
    """Applies on fixed buffers whose sources are rewritten in place.  A graph
    replay starts before the bounding box is known: it stands when the box is
    unchanged (a permutation of the sources) and is redone when the box has
    changed (the sources shifted and shrunk in x).  Every apply equals, bit for
    bit, a plan without graphs on the same points."""
    import torch
    from paper_1902_08250_amd.lmfmm import Plan
    say("speculative replay with moving sources", precision)
    dt = np.complex128 if precision == "c128" else np.complex64
    tol = 1e-10 if precision == "c128" else 1e-6
    pl = Plan(mid["k"], mid["d"], order=16, tol=tol, levels=5)
    ref_pl = Plan(mid["k"], mid["d"], order=16, tol=tol, levels=5)
    ref_pl.set_option("graph", "0")
    s_host = mid["src"].copy()
    src, tgt = dev(s_host), dev(mid["tgt"])
    q = dev(mid["q"][:2].astype(dt))
    u = torch.empty((2, tgt.shape[1]), dtype=q.dtype, device="cuda")
    rng = np.random.default_rng(5)
    for it in range(9):
        if it == 4:
            s_host = np.ascontiguousarray(s_host[:, rng.permutation(s_host.shape[1])])
        if it == 6:
            s_host = s_host.copy()
            s_host[0] = 0.9 * s_host[0] + 0.05
        if it in (4, 6):
            src.copy_(torch.from_numpy(s_host).cuda())
            torch.cuda.synchronize()
        pl.apply(src, q, tgt, out=u)
        got = host(u)
        want = host(ref_pl.apply(dev(s_host), q, tgt))
        assert np.array_equal(got, want), f"apply {it}"
    st = pl.stats()
    say("graph applies", st["graph_applies"])
    assert st["graph_applies"] >= 6
