"""Seeded synthetic inputs for the five workloads (no method arithmetic here).

This module only draws points and densities; it is shared by the tests, the
benchmark and the smoke check, and it neither imports nor is imported by the
GPU binding or the oracle.  There is no public dataset for this method: every
input is drawn from the uniform slab distributions below, with standard normal
real and imaginary density parts.

Draw order for one instance with generator ``numpy.random.default_rng(seed)``:
source x, source y, target x, target y, Re q, Im q, Re w, Im w.
"""
import numpy as np

# (k1, k2, k3, d) of the three-layer medium used by each workload
MEDIUM_A = ((10 + 0.01j, 20 + 0.01j, 15 + 0.01j), 1.0)
MEDIUM_B = ((40 + 0.01j, 60 + 0.01j, 50 + 0.01j), 0.5)

WORKLOADS = {
    0: dict(name="plain-512", n_src=512, n_tgt=512, medium=MEDIUM_A, order=20, levels=3,
            tol=1e-10, precision="c128", x=(0.0, 1.0), ys=(0.05, 1.0), yt=(-0.95, -0.05), nrhs=1),
    1: dict(name="mixed-uniform-1e5", n_src=100_000, n_tgt=100_000, medium=MEDIUM_A, order=16,
            levels=7, tol=1e-6, precision="c64", x=(0.0, 1.0), ys=(0.05, 1.0), yt=(-0.95, -0.05),
            nrhs=1),
    2: dict(name="near-interface-2e5", n_src=200_000, n_tgt=200_000, medium=MEDIUM_B, order=20,
            levels=12, tol=1e-10, precision="c128", x=(0.0, 10.0), ys=(1e-4, 1e-3),
            yt=(-1e-3, -1e-4), nrhs=1),
    4: dict(name="backward-1e6", n_src=1_000_000, n_tgt=1_000_000, medium=MEDIUM_A, order=16,
            levels=9, tol=1e-6, precision="c64", x=(0.0, 1.0), ys=(0.05, 1.0), yt=(-0.95, -0.05),
            nrhs=1),
}


def draw_instance(rng, n_src, n_tgt, x, ys, yt, nrhs=1, dtype=np.complex128):
    """Uniform sources in x-range x, y-range ys; targets in x, yt; N(0,1)+iN(0,1)
    densities q (nrhs, n_src) and upstream weights w (nrhs, n_tgt)."""
    sx = rng.uniform(x[0], x[1], n_src)
    sy = rng.uniform(ys[0], ys[1], n_src)
    tx = rng.uniform(x[0], x[1], n_tgt)
    ty = rng.uniform(yt[0], yt[1], n_tgt)
    qr = rng.standard_normal((nrhs, n_src))
    qi = rng.standard_normal((nrhs, n_src))
    wr = rng.standard_normal((nrhs, n_tgt))
    wi = rng.standard_normal((nrhs, n_tgt))
    src = np.ascontiguousarray(np.stack([sx, sy]))
    tgt = np.ascontiguousarray(np.stack([tx, ty]))
    q = (qr + 1j * qi).astype(dtype)
    w = (wr + 1j * wi).astype(dtype)
    return src, tgt, q, w


def make(config, n_src=None, n_tgt=None, seed=None, nrhs=None):
    """Inputs of one workload, optionally resized (same slabs and medium).
    Returns a dict with src, tgt (float64 (2, n)), q, w (complex (nrhs, n)),
    k (3 complex), d, and the solver settings of the workload."""
    spec = dict(WORKLOADS[config])
    if n_src is not None:
        spec["n_src"] = n_src
    if n_tgt is not None:
        spec["n_tgt"] = n_tgt
    if nrhs is not None:
        spec["nrhs"] = nrhs
    rng = np.random.default_rng(config if seed is None else seed)
    dtype = np.complex128 if spec["precision"] == "c128" else np.complex64
    src, tgt, q, w = draw_instance(rng, spec["n_src"], spec["n_tgt"], spec["x"], spec["ys"], spec["yt"],
                                   spec["nrhs"], dtype)
    k, d = spec["medium"]
    spec.update(src=src, tgt=tgt, q=q, w=w, k=k, d=d)
    return spec


def make_batched(seed=3, n_inst=16, nrhs_per_inst=4, n_lo=1000, n_hi=200_000):
    """Batched workload: n_inst instances, log-uniform N in [n_lo, n_hi] (M = N),
    per-instance k1 ~ U[5,30], k2 ~ U[10,60], k3 ~ U[5,40] (each + 0.01i),
    d ~ U[0.5, 2]; sources in x in [0,1], y in (0.05, 1); targets in
    y in (-0.95 d, -0.05 d).  complex64 densities, nrhs_per_inst each."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n_inst):
        n = int(round(np.exp(rng.uniform(np.log(n_lo), np.log(n_hi)))))
        k1 = rng.uniform(5, 30) + 0.01j
        k2 = rng.uniform(10, 60) + 0.01j
        k3 = rng.uniform(5, 40) + 0.01j
        d = rng.uniform(0.5, 2.0)
        src, tgt, q, w = draw_instance(rng, n, n, (0.0, 1.0), (0.05, 1.0), (-0.95 * d, -0.05 * d),
                                       nrhs_per_inst, np.complex64)
        out.append(dict(src=src, tgt=tgt, q=q, w=w, k=(k1, k2, k3), d=d, n=n))
    return out
