"""Maxwell construction for the equations of state of the oracle (TEST INFRASTRUCTURE).

Coexistence densities (rho_v, rho_l) and pressure p0 satisfy mechanical equilibrium
p(rho_v) = p(rho_l) = p0 and chemical equilibrium, the equal-area rule in the specific volume
1/rho:  integral_{rho_v}^{rho_l} (p(rho) - p0) / rho^2 d rho = 0  (Sec. II.B and Sec. III of the
paper, which use it to fix the spinodal points of Eq. (15)).

Everything here is plain scipy: bracketing root finders and adaptive quadrature.
"""
from __future__ import annotations

import math

import warnings

from scipy import integrate, optimize


def cs_pressure(rho: float, a: float, b: float, R: float, T: float) -> float:
    """Carnahan-Starling: p = rho R T (1 + eta + eta^2 - eta^3)/(1 - eta)^3 - a rho^2, eta = b rho/4."""
    eta = b * rho / 4.0
    return rho * R * T * (1 + eta + eta ** 2 - eta ** 3) / (1 - eta) ** 3 - a * rho ** 2


def _equal_area(p, rv: float, rl: float, p0: float) -> float:
    # substitute rho = exp(s): integral of (p(e^s) - p0) e^{-s} ds, smooth over [ln rv, ln rl]
    with warnings.catch_warnings():
        # near the root the integral itself tends to zero and its relative tolerance is unreachable
        warnings.simplefilter("ignore", integrate.IntegrationWarning)
        val, _ = integrate.quad(lambda s: (p(math.exp(s)) - p0) * math.exp(-s), math.log(rv),
                                math.log(rl), epsabs=0.0, epsrel=1e-13, limit=400)
    return val


def _spinodals(p, lo: float, hi: float, n: int = 4000):
    """Local max and min of p on (lo, hi) located on a grid then refined with Brent's method."""
    h = 1e-7 * hi

    def dp(r):
        return (p(r + h) - p(r - h)) / (2 * h)

    xs = [lo + (hi - lo) * (k + 0.5) / n for k in range(n)]
    ds = [dp(x) for x in xs]
    roots = []
    for k in range(n - 1):
        if ds[k] == 0.0 or (ds[k] > 0) != (ds[k + 1] > 0):
            roots.append(optimize.brentq(dp, xs[k], xs[k + 1], xtol=1e-15, rtol=1e-14))
    if len(roots) != 2:
        raise ValueError("EOS is not in its two-phase (van der Waals loop) regime")
    return roots[0], roots[1]


def maxwell_cs(a: float, b: float, R: float, T: float):
    """(rho_v, rho_l, p0) of the Carnahan-Starling fluid at temperature T (T < T_c)."""
    def p(r):
        return cs_pressure(r, a, b, R, T)

    hi = 4.0 / b * 0.999
    s1, s2 = _spinodals(p, 1e-9, hi)
    pmax, pmin = p(s1), p(s2)

    def branches(p0):
        rv = optimize.brentq(lambda r: p(r) - p0, 1e-300, s1, xtol=1e-300, rtol=1e-15)
        rl = optimize.brentq(lambda r: p(r) - p0, s2, hi, xtol=1e-300, rtol=1e-15)
        return rv, rl

    def area(p0):
        rv, rl = branches(p0)
        return _equal_area(p, rv, rl, p0)

    lo_p = max(pmin, 0.0) * (1 + 1e-12) + 1e-300
    hi_p = pmax * (1 - 1e-12)
    p0 = optimize.brentq(area, lo_p, hi_p, xtol=1e-300, rtol=1e-15, maxiter=500)
    rv, rl = branches(p0)
    return rv, rl, p0


def cs_critical(a: float, b: float, R: float):
    """Critical point of Carnahan-Starling: T_c and rho_c (dp/drho = d2p/drho2 = 0)."""
    # With D1 = d(eta Z)/d eta = (1 + 4e + 4e^2 - 4e^3 + e^4)/(1 - e)^4 and
    # D2 = dD1/d eta = (8 + 20e - 4e^2)/(1 - e)^5, the conditions dp/drho = d2p/drho2 = 0 give
    # D1 = eta D2, i.e. e^5 - 5e^4 + 4e^3 + 20e^2 + 5e - 1 = 0, and R T_c = 8 a / (b D2).
    e = optimize.brentq(lambda e: e ** 5 - 5 * e ** 4 + 4 * e ** 3 + 20 * e ** 2 + 5 * e - 1,
                        0.01, 0.5, xtol=1e-17, rtol=1e-15)
    rho_c = 4 * e / b
    D2 = (8 + 20 * e - 4 * e ** 2) / (1 - e) ** 5
    T_c = 8 * a / (b * R * D2)
    return T_c, rho_c


def cs_temperature_for_ratio(a: float, b: float, R: float, ratio: float) -> float:
    """Temperature at which the Maxwell densities of Carnahan-Starling satisfy rho_l/rho_v = ratio."""
    T_c, _ = cs_critical(a, b, R)

    def g(T):
        rv, rl, _ = maxwell_cs(a, b, R, T)
        return math.log(rl / rv) - math.log(ratio)

    return optimize.brentq(g, 0.3 * T_c, 0.95 * T_c, xtol=1e-15, rtol=1e-14, maxiter=200)


def piecewise_pressure(rho, rho1, rho2, th_v, th_m, th_l):
    """Eq. (15)."""
    if rho <= rho1:
        return rho * th_v
    if rho <= rho2:
        return rho1 * th_v + (rho - rho1) * th_m
    return rho1 * th_v + (rho2 - rho1) * th_m + (rho - rho2) * th_l


def piecewise_spinodals(rho_v, rho_l, th_v, th_m, th_l):
    """(rho1, rho2) of Eq. (15) for given coexistence densities: mechanical equilibrium
    p(rho_v) = p(rho_l) and the equal-area rule (Sec. III)."""
    def eqs(z):
        r1, r2 = z
        p = lambda r: piecewise_pressure(r, r1, r2, th_v, th_m, th_l)  # noqa: E731
        p0 = p(rho_v)
        mech = p(rho_l) - p0
        # equal area; the integrand has kinks at r1 and r2, so integrate piecewise
        chem = 0.0
        pts = [rho_v, r1, r2, rho_l]
        for lo, hi in zip(pts[:-1], pts[1:]):
            with warnings.catch_warnings():
                warnings.simplefilter("ignore", integrate.IntegrationWarning)
                v, _ = integrate.quad(lambda r: (p(r) - p0) / r ** 2, lo, hi, epsabs=0,
                                      epsrel=1e-13, limit=200)
            chem += v
        return [mech, chem]

    # mechanical equilibrium fixes r2 given r1 (linear), leaving one equation for r1
    def r2_of(r1):
        p0 = rho_v * th_v
        # p(rho_l) = r1 th_v + (r2 - r1) th_m + (rho_l - r2) th_l = p0
        return (p0 - r1 * th_v + r1 * th_m - rho_l * th_l) / (th_m - th_l)

    def chem_of(r1):
        return eqs((r1, r2_of(r1)))[1]

    r1 = optimize.brentq(chem_of, rho_v * (1 + 1e-9), 10 * rho_v, xtol=1e-15, rtol=1e-15)
    return r1, r2_of(r1)
