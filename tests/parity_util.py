"""Element-by-element comparison used by the parity tests.

Two figures per comparison, over the compared entries e_i = u_i - ref_i:
  * rel-l2 = ||e||_2 / ||ref||_2, held to the precision's tolerance;
  * the worst entry, max_i |e_i| / max(|ref_i|, rms(ref)) with
    rms(ref) = ||ref||_2 / sqrt(n): the entry's relative error, except that
    entries smaller than the rms are measured against the rms (an entry of a
    random-density field can come arbitrarily close to zero).  It is held to
    PEAK_FACTOR times the same tolerance: rounding- and truncation-type errors
    spread over many entries reach a few times their rms at the largest one,
    which the bound passes, while one bad entry that the norm alone would
    hide fails it.

Tolerances: 1e-10 for the FP64 path and 1e-6 for the mixed path (complex64
densities, FP32 expansions), the figures the method is specified to meet.
"""
import numpy as np

TOL = {"c128": 1e-10, "c64": 1e-6}
PEAK_FACTOR = 4.0


def errors(u, ref):
    u = np.asarray(u, dtype=np.complex128).ravel()
    ref = np.asarray(ref, dtype=np.complex128).ravel()
    e = np.abs(u - ref)
    nrm = np.linalg.norm(ref)
    rms = nrm / np.sqrt(ref.size)
    return float(np.linalg.norm(u - ref) / nrm), float(np.max(e / np.maximum(np.abs(ref), rms)))


def check(u, ref, tol, label="", say=print):
    rl2, peak = errors(u, ref)
    say(f"{label}: rel-l2 {rl2:.3e}, worst entry {peak:.3e} (tol {tol:g}, worst-entry bound {PEAK_FACTOR * tol:g})")
    assert rl2 < tol, f"{label}: rel-l2 {rl2} >= {tol}"
    assert peak < PEAK_FACTOR * tol, f"{label}: worst entry {peak} >= {PEAK_FACTOR * tol}"
    return rl2, peak
