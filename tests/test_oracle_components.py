"""Pins of the oracle's other field components (Section 3, Examples 3 and 4):
g_1^s (top layer), g_2^b (middle layer, from the bottom interface), g_3^s
(bottom layer) and the impedance half-space.  Nothing here retypes the
oracle's formulas; each component is held to something the paper or the
mathematics fixes:

  * the densities against the paper's 4x4 interface system, solved by numpy
    (its unknowns are sigma_1, sigma_2^t, e^{-d s2} sigma_2^b, e^{-d s3}
    sigma_3 of the closed forms);
  * a homogeneous medium (k1 = k2 = k3): no reflected parts (g_1^s = g_2^b =
    0) and the free field (i/4) H0(k r) transmitted to the bottom layer;
  * the transmission conditions: the total field (the free field of the
    source plus g_1^s above y = 0, g_2^t + g_2^b between, g_3^s below y = -d)
    and its y-derivative are continuous across both interfaces;
  * the impedance half-space: alpha = 0 gives the image source (i/4)
    H0(k |x - x0'|), x0' = (x0, -y0); alpha -> infinity its negative; and the
    total field meets u_y + i k alpha u = 0 on y = 0 (the condition that the
    printed image term (s + i k alpha)/(s - i k alpha) satisfies; the text's
    u_y - i alpha u = 0 differs in sign and in the factor k).
"""
import numpy as np
import pytest
from scipy.special import hankel1

K = (10 + 0.01j, 20 + 0.01j, 15 + 0.01j)
D = 1.0
SRC = (0.13, 0.41)


def sroot(lam, k):
    z = np.sqrt(lam * lam - k * k + 0j)
    return np.where(z.real < 0, -z, z)


def free(x, y, x0, y0, k):
    """(i/4) H0(k r) and its y-derivative."""
    r = np.hypot(x - x0, y - y0)
    return 0.25j * hankel1(0, k * r), -0.25j * k * hankel1(1, k * r) * (y - y0) / r


def test_densities_solve_the_interface_system(orc):
    rng = np.random.default_rng(41)
    lam = rng.uniform(-40, 40, 12) + 1j * rng.uniform(-3, 3, 12)
    s = {c: orc.sigma(lam, K, D, comp=c) for c in ("1s", "2t", "2b", "3s")}
    for i, l in enumerate(lam):
        s1, s2, s3 = sroot(l, K[0]), sroot(l, K[1]), sroot(l, K[2])
        e = np.exp(-D * s2)
        A = np.array([[-1, s1 / s2, e * s1 / s2, 0], [0, e, 1, -s2 / s3], [1, 1, -e, 0], [0, e, -1, -1]])
        x = np.linalg.solve(A, np.array([1, 0, 1, 0], dtype=complex))
        got = np.array([s["1s"][i], s["2t"][i], np.exp(-D * s2) * s["2b"][i], np.exp(-D * s3) * s["3s"][i]])
        assert np.allclose(got, x, rtol=1e-11, atol=1e-13 * np.abs(x).max()), (l, got, x)


def test_homogeneous_medium(orc):
    k = 12 + 0.01j
    kk = (k, k, k)
    x0, y0 = SRC
    for (x, y) in ((0.5, -1.3), (0.1, -1.05), (2.0, -3.0)):
        g3 = orc.entry(x, y, x0, y0, kk, D, comp="3s")
        ref, _ = free(x, y, x0, y0, k)
        assert abs(g3 - ref) < 1e-12 * abs(ref)
    # (the reflected densities vanish identically, so g_1^s = g_2^b = 0; their
    # entries are not evaluated: the adaptive quadrature of an integrand that
    # is rounding noise has no scale to converge to)
    lam = np.linspace(-30, 30, 7) + 0.5j
    assert np.max(np.abs(orc.sigma(lam, kk, D, comp="1s"))) < 1e-13
    assert np.max(np.abs(orc.sigma(lam, kk, D, comp="2b"))) < 1e-13
    assert np.max(np.abs(orc.sigma(lam, kk, D, comp="3s") - 1)) < 1e-13


def limit(fn, y, side, eps=1e-6):
    """Value and y-derivative at the interface y from one side (side = +1 from
    above, -1 from below): linear extrapolation from y + side eps and y + 2 side eps."""
    a = np.array(fn(y + side * eps))
    b = np.array(fn(y + 2 * side * eps))
    return 2 * a - b


@pytest.mark.parametrize("x", [0.13, 0.6, -0.7])
def test_transmission_conditions(orc, x):
    x0, y0 = SRC

    def comp(c, y):
        g = orc.entry(x, y, x0, y0, K, D, comp=c, derivs=True)
        return np.array([g[0], g[2]])  # value, d/dy

    def layer1(y):
        f, fy = free(x, y, x0, y0, K[0])
        return np.array([f, fy]) + comp("1s", y)

    def layer2(y):
        return comp("2t", y) + comp("2b", y)

    def layer3(y):
        return comp("3s", y)

    top_above, top_below = limit(layer1, 0.0, +1), limit(layer2, 0.0, -1)
    bot_above, bot_below = limit(layer2, -D, +1), limit(layer3, -D, -1)
    print("y=0:", top_above, top_below, " y=-d:", bot_above, bot_below)
    for a, b in ((top_above, top_below), (bot_above, bot_below)):
        assert abs(a[0] - b[0]) < 1e-8 * abs(a[0])
        assert abs(a[1] - b[1]) < 1e-7 * max(abs(a[1]), abs(a[0]))


def test_impedance_half_space(orc):
    k = 6 + 0.01j
    kk = (k, k, k)
    x0, y0 = SRC
    for (x, y) in ((0.5, 0.3), (1.5, 0.05), (0.13, 0.9)):
        img, _ = free(x, y, x0, -y0, k)
        g0 = orc.entry(x, y, x0, y0, kk, D, comp="imp", alpha=0.0)
        assert abs(g0 - img) < 1e-12 * abs(img)
        ginf = orc.entry(x, y, x0, y0, kk, D, comp="imp", alpha=1e10)
        assert abs(ginf + img) < 1e-9 * abs(img)
    # u_y + i k alpha u = 0 on y = 0 for the total field u = free + g
    for alpha in (0.3, 1.0, 4.0):
        for x in (0.2, 1.1):
            def total(y):
                g = orc.entry(x, y, x0, y0, kk, D, comp="imp", alpha=alpha, derivs=True)
                f, fy = free(x, y, x0, y0, k)
                return np.array([f + g[0], fy + g[2]])
            u, uy = limit(total, 0.0, +1)
            assert abs(uy + 1j * k * alpha * u) < 1e-7 * abs(uy)
