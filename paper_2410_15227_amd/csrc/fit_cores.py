"""Fit the binary32 polynomial cores of the mixed-precision transcendental
functions in exact.hip (atan_mixed, asinh_mixed, log_ratio_mixed).

Method: discrete minimax of the relative error by linear programming.  On a
dense grid of the reduced argument the coefficients c and a bound e solve
    minimise e  subject to  |sum_j c_j phi_j(x_k) - g(x_k)| <= e |f(x_k)|,
which is the Chebyshev (minimax) approximation on the grid; the LP is solved
with scipy's HiGHS.  The coefficients are then rounded to binary32 and the
whole core is evaluated as the device does (binary32 Horner with fused
multiply-adds, binary64 assembly) to report the achieved relative error of
the function itself.

  atan:  atan(s) = s + s^3 P(s^2) on |s| <= tan(pi/8) (the reduced range
         after the octant reduction), P of degree 5;
  atanh: 2 atanh(t) = 2 t + t^3 Q(t^2) on |t| <= 3 - 2 sqrt(2) (the range
         left by splitting off the binary exponent and folding the mantissa
         into [1/sqrt(2), sqrt(2)]), Q of degree 3; log and asinh use it.

Run: python fit_cores.py   (prints the coefficients in the order Horner
evaluates them, highest degree first, and the achieved errors)."""
from __future__ import annotations

import numpy as np
from scipy.optimize import linprog

TAN_PI_8 = np.tan(np.pi / 8)
ATANH_T = 3.0 - 2.0 * np.sqrt(2.0)


def minimax(z, target, weight, degree):
    """Coefficients a_0..a_degree of p(z) = sum a_j z^j minimising
    max_k |p(z_k) - target_k| / weight_k on the grid z."""
    # rows scaled so that the optimal residuals are of order one (the
    # solver's feasibility tolerance is absolute, about 1e-7)
    scale = 1e9
    A = np.vander(z, degree + 1, increasing=True) / weight[:, None] * scale
    b = target / weight * scale
    n = degree + 1
    # variables: a_0..a_degree, e; minimise e
    c = np.zeros(n + 1)
    c[-1] = 1.0
    A_ub = np.vstack([np.hstack([A, -np.ones((len(z), 1))]), np.hstack([-A, -np.ones((len(z), 1))])])
    b_ub = np.concatenate([b, -b])
    res = linprog(c, A_ub=A_ub, b_ub=b_ub, bounds=[(None, None)] * n + [(0, None)], method="highs")
    assert res.success, res.message
    return res.x[:n], res.x[-1] / scale


def fmaf(a, b, c):
    """binary32 fused multiply-add (the product of two binary32 numbers is
    exact in binary64; one rounding of the sum to binary32)."""
    return np.float32(np.float64(a) * np.float64(b) + np.float64(c))


def horner32(coef_hi_first, zf):
    p = np.float32(coef_hi_first[0]) * np.ones_like(zf)
    for c in coef_hi_first[1:]:
        p = fmaf(p, zf, np.float32(c))
    return p


def atan_core(P32, s):
    """s + s^3 P(s^2): s, z = s^2 and the assembly in binary64, P in binary32."""
    z = s * s
    P = horner32(P32, z.astype(np.float32)).astype(np.float64)
    return s + (s * z) * P


def atanh2_core(Q32, t):
    """2 atanh(t) = 2t + t^3 Q(t^2), Q in binary32."""
    t2 = t * t
    Q = horner32(Q32, t2.astype(np.float32)).astype(np.float64)
    return 2.0 * t + (t * t2) * Q


def fit_atan(degree=5, n=20000):
    s = np.linspace(1e-6, TAN_PI_8, n)
    z = s * s
    # (atan(s) - s) / s^3 = P(z); relative error of atan: s^3 |P - P*| / atan(s)
    target = (np.arctan(s) - s) / (s * z)
    weight = np.arctan(s) / (s * z)
    a, e = minimax(z, target, weight, degree)
    return a[::-1].astype(np.float32), e


def fit_atanh(degree=3, n=20000):
    t = np.linspace(1e-6, ATANH_T, n)
    t2 = t * t
    f = 2.0 * np.arctanh(t)
    target = (f - 2.0 * t) / (t * t2)
    weight = f / (t * t2)
    a, e = minimax(t2, target, weight, degree)
    return a[::-1].astype(np.float32), e


def achieved(P32, Q32, n=200001):
    s = np.linspace(-TAN_PI_8, TAN_PI_8, n)
    s = s[s != 0]
    ea = np.max(np.abs(atan_core(P32, s) - np.arctan(s)) / np.abs(np.arctan(s)))
    t = np.linspace(-ATANH_T, ATANH_T, n)
    t = t[t != 0]
    eh = np.max(np.abs(atanh2_core(Q32, t) - 2.0 * np.arctanh(t)) / np.abs(2.0 * np.arctanh(t)))
    return ea, eh


if __name__ == "__main__":
    P, e1 = fit_atan()
    Q, e2 = fit_atanh()
    print("atan  P (highest degree first):", ", ".join(f"{float(c)!r}f" for c in P), f"  (LP bound {e1:.2e})")
    print("atanh Q (highest degree first):", ", ".join(f"{float(c)!r}f" for c in Q), f"  (LP bound {e2:.2e})")
    ea, eh = achieved(P, Q)
    print(f"achieved relative error with binary32 coefficients: atan {ea:.2e}, 2 atanh {eh:.2e}")
