"""The weighted straight-line fit of Section 6 ("Linear fit"), from its
definition, in mpmath.  TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Section 6 writes the leading-order asymptotics of lambda_1(N) as a line
y = a + b x, x = log(4 pi N e), y = log(8 pi sqrt(log N) / lambda_1(N)), whose
slope b is the leading exponent 2/pi, and fits a and b by least squares with
each point weighted proportionally to N^2.  Here the fit is the textbook closed
form of weighted least squares (weighted means, centred sums of squares), the
residual variance sum w r^2 / (n - 2), the standard errors that follow from it,
and two-sided Student-t intervals whose quantile is found by bisection on the
t distribution function written through the regularised incomplete beta
function.

Parity status: pinned in tests/test_exponent_fit.py by the numbers Section 6
prints for the lambda_1 of Table 2 (slope, intercept, adjusted R-squared, the
interval), by exact recovery of a line, and by textbook t quantiles.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import Sequence, Tuple

import mpmath


@dataclass
class Line:
    intercept: object
    slope: object
    se_intercept: object
    se_slope: object
    r2: object
    adj_r2: object
    residuals: list
    dof: int


def xy(N: int, lam1, prec: int = 200) -> Tuple[object, object]:
    """The coordinates of Section 6: x = log(4 pi N e), y = log(8 pi sqrt(log N) / lambda_1)."""
    with mpmath.workprec(prec):
        x = mpmath.log(4 * mpmath.pi * N * mpmath.e)
        y = mpmath.log(8 * mpmath.pi * mpmath.sqrt(mpmath.log(N)) / mpmath.mpf(lam1))
        return x, y


def line(Ns: Sequence[int], lam1s: Sequence, weight_power: int = 2, prec: int = 200) -> Line:
    """Weighted least squares of y on x with weights N^weight_power."""
    with mpmath.workprec(prec):
        pts = [xy(N, l, prec) for N, l in zip(Ns, lam1s)]
        w = [mpmath.mpf(N) ** weight_power for N in Ns]
        W = mpmath.fsum(w)
        xb = mpmath.fsum(wi * p[0] for wi, p in zip(w, pts)) / W
        yb = mpmath.fsum(wi * p[1] for wi, p in zip(w, pts)) / W
        sxx = mpmath.fsum(wi * (p[0] - xb) ** 2 for wi, p in zip(w, pts))
        sxy = mpmath.fsum(wi * (p[0] - xb) * (p[1] - yb) for wi, p in zip(w, pts))
        syy = mpmath.fsum(wi * (p[1] - yb) ** 2 for wi, p in zip(w, pts))
        b = sxy / sxx
        a = yb - b * xb
        res = [p[1] - a - b * p[0] for p in pts]
        n = len(pts)
        ssr = mpmath.fsum(wi * r * r for wi, r in zip(w, res))
        s2 = ssr / (n - 2)
        r2 = 1 - ssr / syy
        return Line(intercept=a, slope=b, se_intercept=mpmath.sqrt(s2 * (1 / W + xb * xb / sxx)),
                    se_slope=mpmath.sqrt(s2 / sxx), r2=r2, adj_r2=1 - (1 - r2) * (n - 1) / (n - 2),
                    residuals=res, dof=n - 2)


def t_cdf(t, nu: int, prec: int = 200):
    """Student-t distribution function: for t >= 0, 1 - I_{nu/(nu+t^2)}(nu/2, 1/2) / 2."""
    with mpmath.workprec(prec):
        t = mpmath.mpf(t)
        tail = mpmath.betainc(mpmath.mpf(nu) / 2, mpmath.mpf(1) / 2, 0, nu / (nu + t * t), regularized=True) / 2
        return 1 - tail if t >= 0 else tail


def t_quantile(p, nu: int, prec: int = 200, bits: int = 120):
    """The t with t_cdf(t) = p (1/2 < p < 1), by bisection."""
    with mpmath.workprec(prec):
        lo, hi = mpmath.mpf(0), mpmath.mpf(1)
        while t_cdf(hi, nu, prec) < p:
            hi *= 2
        for _ in range(bits):
            mid = (lo + hi) / 2
            if t_cdf(mid, nu, prec) < p:
                lo = mid
            else:
                hi = mid
        return (lo + hi) / 2


def interval(fit: Line, level, prec: int = 200):
    """Two-sided Student-t interval for the slope at confidence ``level``."""
    with mpmath.workprec(prec):
        q = t_quantile((1 + mpmath.mpf(str(level))) / 2, fit.dof, prec)
        return fit.slope - q * fit.se_slope, fit.slope + q * fit.se_slope
