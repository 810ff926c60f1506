"""Pins of the oracle's kernel pieces against mathematics that does not go
through the oracle: the M4 cubic spline truncated at 2h (Sec. 2.4.2) with the
3-D normalisation 1/(pi h^3)."""
import math

import numpy as np
import pytest
from scipy import integrate

pytestmark = pytest.mark.filterwarnings("ignore")


def m4(q):
    q = np.asarray(q, float)
    return np.where(q < 1, 1 - 1.5 * q**2 + 0.75 * q**3, np.where(q < 2, 0.25 * (2 - q) ** 3, 0.0))


def test_phi_is_cumulative_kernel_mass(oracle):
    # Phi(q) = 4 int_0^q s^2 w(s) ds by adaptive quadrature of the kernel itself
    for q in [0.1, 0.5, 0.99, 1.0, 1.3, 1.7, 1.999, 2.0, 2.5]:
        ref, _ = integrate.quad(lambda s: 4 * s * s * m4(s), 0, q, points=[1.0] if q > 1 else None,
                                epsabs=1e-14, epsrel=1e-14)
        assert abs(oracle.Phi(q) - ref) < 1e-13, q
    assert abs(oracle.Phi(1.0) - 19.0 / 30.0) < 1e-15
    assert oracle.Phi(2.0) == 1.0


def test_kernel_normalised(oracle):
    # int W dV over R^3 = 1 with W = w(r/h)/(pi h^3), h = 1
    tot, _ = integrate.quad(lambda r: 4 * math.pi * r * r * m4(r) / math.pi, 0, 2, points=[1.0])
    assert abs(tot - 1.0) < 1e-13


def test_G_is_antiderivative(oracle):
    # G'(u) = Phi(u)/u^2 (central differences) and G continuous across 1 and 2
    for u in [0.05, 0.4, 0.9, 1.2, 1.6, 1.95, 2.4, 5.0]:
        e = 1e-6 * u
        num = (oracle.G(u + e) - oracle.G(u - e)) / (2 * e)
        assert abs(num - oracle.Phi(u) / (u * u)) < 1e-7 * max(1.0, 1.0 / u**2), u
    for k in [1.0, 2.0]:
        assert abs(oracle.G(k * (1 - 1e-15)) - oracle.G(k)) < 1e-13


def test_psi_radial_integral(oracle):
    # Psi_d(U) = |d| int_{|d|}^{U} Phi(u)/u^2 du, Phi from quadrature of the kernel
    def phi_ref(u):
        return integrate.quad(lambda s: 4 * s * s * m4(s), 0, min(u, 2.0), points=[1.0] if u > 1 else None,
                              epsabs=1e-14)[0]

    for ad, U in [(0.2, 0.9), (0.2, 1.7), (0.7, 2.6), (1.3, 1.9), (2.2, 3.0), (0.05, 0.06)]:
        ref, _ = integrate.quad(lambda u: phi_ref(u) / (u * u), ad, U, points=[p for p in (1.0, 2.0) if ad < p < U],
                                epsabs=1e-13)
        assert abs(oracle.Psi(ad, U) - ad * ref) < 1e-11, (ad, U)


def test_fan_full_mass_beyond_support(oracle):
    # beyond 2h every direction holds the whole kernel: the fan integral is the
    # solid-angle integrand 1 - |d|/U, whose integral is phi - atan(|d| tan(phi)/U)
    ad, p = 2.3, 0.8
    pa, pb = -0.4, 0.9
    ref = 0.0
    for ph in (pb, pa):
        U = math.sqrt(ad * ad + p * p / math.cos(ph) ** 2)
        ref += (1 if ph == pb else -1) * (ph - math.atan(ad * math.tan(ph) * abs(p) / (abs(p) * U)))
    # the atan form above is the closed solid-angle integral of a right triangle
    assert abs(oracle.fan_integral(ad, p, pa, pb) - ref) < 1e-12
