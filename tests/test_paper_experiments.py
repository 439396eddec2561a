"""The paper's own numerical experiments (Section 5), reproduced on the CPU
with numpy/scipy quadrature (independent of the GPU library and the oracle):

  * Fig. 3: Gauss-Legendre nodes needed on the finite segment IV of the
    impedance half-space's evanescent integral (x = 1, y = 0.1, k = 1,
    c = 2): about 17 on the first contour, about 200 on the second (the text's
    figures; the impedance alpha is not stated: alpha = 1 reproduces them);
  * Fig. 4: the term ratio |J_{p+1} Phi_{p+1}| / |J_p Phi_p| of the multipole
    expansion of the impedance half-space (x - x_c = 2, y + y_c = 3, r = 1.5,
    k = 0.1, alpha = 1) tends to r / rho with the modified distance
    rho = sqrt(2^2 + 3^2);
  * Fig. 5 (Theorem 1): the same for the local expansion of the three-layer
    g_2^t (k = (1, 3, 1), x0 - x_c = 2, y0 - y_c = 3, r = 1.5): the ratio
    tends to r / rho = 1.5 / sqrt(13) = 0.416.  The printed rho = sqrt(2^2 + 3^3)
    is read as sqrt(2^2 + 3^2), the value the text states (0.416); d is not
    given and the limit does not depend on it (d = 1 here);
  * Remark after Theorem 1: with the modified distance the multipole
    expansion also converges for a target in the source box itself.
"""
import numpy as np
import pytest
from scipy.integrate import quad
from scipy.special import jv

R_OVER_RHO = 1.5 / np.sqrt(13.0)


def gl(f, n, lo, hi):
    x, w = np.polynomial.legendre.leggauss(n)
    t = lo + 0.5 * (hi - lo) * (x + 1.0)
    return 0.5 * (hi - lo) * np.sum(w * f(t))


def nodes_needed(f, lo, hi, tol, nmax=400):
    ref = gl(f, 2000, lo, hi)
    for n in range(2, nmax):
        if abs(gl(f, n, lo, hi) - ref) <= tol * abs(ref):
            return n
    return nmax


def test_fig3_first_contour_needs_far_fewer_nodes():
    x, y, k, c, alpha = 1.0, 0.1, 1.0, 2.0, 1.0

    def first(t):  # segment IV of the first contour, t in [0, c]
        r = np.sqrt(t * t + k * k)
        return np.exp(-t * y) * np.exp(1j * x * r) / r * (t + 1j * alpha) / (t - 1j * alpha)

    r, th = np.hypot(x, y), np.arctan2(y, x)

    def second(u):  # segment IV of the second contour, u in [0, 1]
        psi = (c + 1j * np.cos(th)) * u - 1j * np.cos(th)
        sq = np.sqrt(1.0 + psi * psi)
        phi = 1j * k * np.cos(th) * sq + psi * k * np.sin(th)
        return np.exp(-k * r * psi) / sq * (phi + 1j * alpha) / (phi - 1j * alpha) * (c + 1j * np.cos(th))

    n1 = nodes_needed(first, 0.0, c, 1e-12)
    n2 = nodes_needed(second, 0.0, 1.0, 1e-12)
    print("Gauss-Legendre nodes for 1e-12: first contour", n1, "second contour", n2)
    assert n1 <= 20
    assert n2 >= 120


def ratio_sequence(basis, k, r, ps):
    vals = {p: basis(p) for p in range(ps[0], ps[-1] + 2)}
    return {p: abs(jv(p + 1, k * r) * vals[p + 1]) / abs(jv(p, k * r) * vals[p]) for p in ps}


def cquad(f, a, b):
    re = quad(lambda t: f(t).real, a, b, limit=800, epsabs=0, epsrel=1e-11)[0]
    im = quad(lambda t: f(t).imag, a, b, limit=800, epsabs=0, epsrel=1e-11)[0]
    return re + 1j * im


def sroot(lam, k):
    z = np.sqrt(complex(lam * lam - k * k))
    return z if z.real >= 0 else -z


@pytest.mark.filterwarnings("ignore::scipy.integrate.IntegrationWarning")
def test_fig4_impedance_multipole_ratio():
    k, alpha, X, Y, r = 0.1, 1.0, 2.0, 3.0, 1.5

    def phi(p):  # evanescent part of the multipole basis, lam in (k, inf)
        def f(lam):
            s = sroot(lam, k)
            sig = (s + 1j * k * alpha) / (s - 1j * k * alpha)
            return ((lam + s) / k) ** p * np.exp(-s * Y + 1j * lam * X) * sig / (4 * np.pi * s)
        return cquad(f, k, k + 200 + 5 * p)

    R = ratio_sequence(phi, k, r, [30, 40, 50, 60])
    print("impedance term ratios", R, "r/rho", R_OVER_RHO)
    for p in (40, 50, 60):
        assert abs(R[p] - R_OVER_RHO) < 0.02


@pytest.mark.filterwarnings("ignore::scipy.integrate.IntegrationWarning")
def test_fig5_three_layer_local_ratio():
    k1, k2, k3, d = 1.0, 3.0, 1.0, 1.0
    X, Y, r, y0 = 2.0, 3.0, 1.5, 3.5

    def sig2t(lam):
        s1, s2, s3 = sroot(lam, k1), sroot(lam, k2), sroot(lam, k3)
        e = np.exp(-2 * d * s2)
        num = lam * lam + s2 * s3 - k2 * k2
        den = 0.5 * (1 - e) * (lam * lam + s1 * s3 - k2 * k2) + 0.5 * s2 * (s1 + s3) * (1 + e)
        return num / den

    def psi(p):  # evanescent part of the local basis, lam in (k2, inf)
        def f(lam):
            s1, s2 = sroot(lam, k1), sroot(lam, k2)
            return ((lam + s2) / k2) ** p * np.exp(-s2 * Y + 1j * lam * X) * np.exp((s2 - s1) * y0) * sig2t(lam) / (
                4 * np.pi * s2)
        return cquad(f, k2, k2 + 200 + 5 * p)

    R = ratio_sequence(psi, k2, r, [5, 30, 40, 50, 60])
    print("three-layer term ratios", R, "r/rho", R_OVER_RHO)
    assert R[5] > 0.6  # far from the limit at low order
    for p in (40, 50, 60):
        assert abs(R[p] - R_OVER_RHO) < 0.02
    # the printed rho = sqrt(2^2 + 3^3) would give 0.269
    assert abs(R[60] - 1.5 / np.sqrt(31.0)) > 0.1


@pytest.mark.filterwarnings("ignore::scipy.integrate.IntegrationWarning")
def test_multipole_valid_in_own_box_under_modified_distance():
    """Remark after Theorem 1: the scattered field's multipole expansion can
    converge in the source box itself.  Source box centre and target both at
    (0, 1.5), so the physical distance is 0, while the modified distance is
    y + y_c = 3: the term ratio of the impedance half-space's expansion
    tends to r / 3 = 0.5 < 1.  The imaged tree places such a target at
    (0, -1.5), at twice the radius r from the source centre, so the pair is a far
    pair there."""
    k, alpha, y, yc, r = 0.1, 1.0, 1.5, 1.5, 1.5

    def phi(p):
        def f(lam):
            s = sroot(lam, k)
            sig = (s + 1j * k * alpha) / (s - 1j * k * alpha)
            return ((lam + s) / k) ** p * np.exp(-s * (y + yc)) * sig / (4 * np.pi * s)
        return cquad(f, k, k + 200 + 5 * p)

    R = ratio_sequence(phi, k, r, [40, 50, 60])
    print("own-box term ratios", R, "r/(y+yc)", r / (y + yc))
    for p in (40, 50, 60):
        assert abs(R[p] - r / (y + yc)) < 0.02
