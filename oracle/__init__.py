"""Test infrastructure only: the FP64 CPU oracle for applying g_2^t.

Plain O(N*M) direct sums in which every kernel entry is an adaptive
Sommerfeld quadrature (``lmfmm_oracle.c``).  Only the test suite,
``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py`` may use
this package; the GPU library never imports it and shares no code with it.

Conventions (same as the GPU library's C ABI so results compare directly):
  * coordinates are float64 SoA arrays of shape (2, n): row 0 = x, row 1 = y;
  * densities are complex128 arrays of shape (nrhs, n);
  * the medium is (k1, k2, k3, d) with complex wave numbers (Im k >= 0).
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lmfmm_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force=True):
    """Compile the oracle with gcc + OpenMP into oracle/liboracle.so."""
    cmd = ["gcc", "-O2", "-fopenmp", "-std=c99", "-D_GNU_SOURCE", "-shared", "-fPIC",
           _SRC, "-o", _LIB, "-lm"]
    if force or not os.path.exists(_LIB):
        subprocess.check_call(cmd)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build(force=False)
    lib = ctypes.CDLL(_LIB)
    D = ctypes.POINTER(ctypes.c_double)
    L = ctypes.c_long
    I = ctypes.c_int
    lib.orc_sigma2t.argtypes = [D, I, L, D, D]
    lib.orc_sigma.argtypes = [D, I, L, D, D]
    lib.orc_entry.argtypes = [D, I, D, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                              ctypes.c_double, I, D, ctypes.POINTER(I)]
    lib.orc_apply.argtypes = [D, I, D, L, D, D, L, D, D, I, I]
    lib.orc_apply_adjoint.argtypes = [D, I, D, L, D, L, D, D, D, I, I]
    lib.orc_grad_coords.argtypes = [D, I, D, L, D, D, L, D, D, I, D, D, I]
    lib.orc_max_threads.argtypes = []
    for f in (lib.orc_sigma2t, lib.orc_sigma, lib.orc_entry, lib.orc_apply, lib.orc_apply_adjoint,
              lib.orc_grad_coords, lib.orc_max_threads):
        f.restype = I
    _lib = lib
    return lib


class OracleError(RuntimeError):
    pass


def _ptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


# field components (the target's layer and part; see lmfmm_oracle.c)
COMP = {"2t": 0, "2b": 1, "1s": 2, "3s": 3, "imp": 4}


def _med(k, d, alpha=0.0):
    k1, k2, k3 = (complex(v) for v in k)
    return np.array([k1.real, k1.imag, k2.real, k2.imag, k3.real, k3.imag, float(d), float(alpha)],
                    dtype=np.float64)


def _flags(sigma_unity=False, comp="2t"):
    return int(bool(sigma_unity)) | (COMP[comp] << 1)


def _opt(eta=1.0, c_factor=1.5, rep=0, eps=1e-15):
    return np.array([eta, c_factor, float(rep), eps], dtype=np.float64)


def _check(rc, what):
    if rc != 0:
        raise OracleError(f"{what} failed with status {rc}")


def max_threads():
    return _load().orc_max_threads()


def sigma2t(lam, k, d, sigma_unity=False):
    """sigma_2^t at complex points lam (any shape)."""
    lib = _load()
    lam = np.ascontiguousarray(np.asarray(lam, dtype=np.complex128))
    flat = lam.reshape(-1)
    out = np.empty_like(flat)
    _check(lib.orc_sigma2t(_ptr(_med(k, d)), _flags(sigma_unity), flat.size,
                           _ptr(flat.view(np.float64)), _ptr(out.view(np.float64))), "sigma2t")
    return out.reshape(lam.shape)


def sigma(lam, k, d, comp="2t", alpha=0.0):
    """The density of component comp ("2t", "2b", "1s", "3s" of the three-layer
    medium; "imp": the impedance half-space with k = k[0]) at complex points lam."""
    lib = _load()
    lam = np.ascontiguousarray(np.asarray(lam, dtype=np.complex128))
    flat = lam.reshape(-1)
    out = np.empty_like(flat)
    _check(lib.orc_sigma(_ptr(_med(k, d, alpha)), _flags(False, comp), flat.size,
                         _ptr(flat.view(np.float64)), _ptr(out.view(np.float64))), "sigma")
    return out.reshape(lam.shape)


def entry(x1, y1, x0, y0, k, d, *, derivs=False, sigma_unity=False, rep=0, eta=1.0,
          c_factor=1.5, eps=1e-15, comp="2t", alpha=0.0):
    """g(x1,y1; x0,y0) of component comp (default g_2^t).  With derivs=True returns
    (g, dg/dx1, dg/dy1, dg/dx0, dg/dy0).
    rep: 0 automatic, 1 north (real-axis tails), 2 east (alternative direction)."""
    lib = _load()
    n = 5 if derivs else 1
    out = np.zeros(n, dtype=np.complex128)
    used = ctypes.c_int(0)
    rc = lib.orc_entry(_ptr(_med(k, d, alpha)), _flags(sigma_unity, comp), _ptr(_opt(eta, c_factor, rep, eps)),
                       float(x1), float(y1), float(x0), float(y0), n, _ptr(out.view(np.float64)),
                       ctypes.byref(used))
    _check(rc, "entry")
    return tuple(out) if derivs else out[0]


def _prep_xy(xy):
    xy = np.ascontiguousarray(np.asarray(xy, dtype=np.float64))
    if xy.ndim != 2 or xy.shape[0] != 2:
        raise ValueError("coordinates must have shape (2, n)")
    return xy


def _prep_dens(q, n):
    q = np.asarray(q, dtype=np.complex128)
    if q.ndim == 1:
        q = q[None, :]
    q = np.ascontiguousarray(q)
    if q.shape[1] != n:
        raise ValueError("density length does not match the point count")
    return q


def apply(src, q, tgt, k, d, *, sigma_unity=False, rep=0, eta=1.0, c_factor=1.5, eps=1e-15,
          threads=0, comp="2t", alpha=0.0):
    """u[r, i] = sum_j g(tgt_i, src_j) q[r, j] for component comp (default g_2^t);
    returns shape (nrhs, n_tgt)."""
    lib = _load()
    src, tgt = _prep_xy(src), _prep_xy(tgt)
    q = _prep_dens(q, src.shape[1])
    u = np.zeros((q.shape[0], tgt.shape[1]), dtype=np.complex128)
    rc = lib.orc_apply(_ptr(_med(k, d, alpha)), _flags(sigma_unity, comp), _ptr(_opt(eta, c_factor, rep, eps)),
                       src.shape[1], _ptr(src), _ptr(q.view(np.float64)), tgt.shape[1], _ptr(tgt),
                       _ptr(u.view(np.float64)), q.shape[0], int(threads))
    _check(rc, "apply")
    return u


def apply_adjoint(src, tgt, w, k, d, *, sigma_unity=False, eps=1e-15, threads=0, comp="2t", alpha=0.0):
    """v[r, j] = sum_i g(tgt_i, src_j) w[r, i]  (transpose, no conjugation)."""
    lib = _load()
    src, tgt = _prep_xy(src), _prep_xy(tgt)
    w = _prep_dens(w, tgt.shape[1])
    v = np.zeros((w.shape[0], src.shape[1]), dtype=np.complex128)
    rc = lib.orc_apply_adjoint(_ptr(_med(k, d, alpha)), _flags(sigma_unity, comp), _ptr(_opt(eps=eps)), src.shape[1],
                               _ptr(src), tgt.shape[1], _ptr(tgt), _ptr(w.view(np.float64)),
                               _ptr(v.view(np.float64)), w.shape[0], int(threads))
    _check(rc, "apply_adjoint")
    return v


def grad_coords(src, q, tgt, w, k, d, *, eps=1e-15, threads=0, comp="2t", alpha=0.0):
    """Gradients of L = Re sum w*u with respect to source and target coordinates.
    Returns (dsrc (2, n_src), dtgt (2, n_tgt))."""
    lib = _load()
    src, tgt = _prep_xy(src), _prep_xy(tgt)
    q = _prep_dens(q, src.shape[1])
    w = _prep_dens(w, tgt.shape[1])
    if q.shape[0] != w.shape[0]:
        raise ValueError("q and w must have the same number of right-hand sides")
    dsrc = np.zeros((2, src.shape[1]))
    dtgt = np.zeros((2, tgt.shape[1]))
    rc = lib.orc_grad_coords(_ptr(_med(k, d, alpha)), _flags(False, comp), _ptr(_opt(eps=eps)), src.shape[1], _ptr(src),
                             _ptr(q.view(np.float64)), tgt.shape[1], _ptr(tgt),
                             _ptr(w.view(np.float64)), q.shape[0], _ptr(dsrc), _ptr(dtgt), int(threads))
    _check(rc, "grad_coords")
    return dsrc, dtgt
