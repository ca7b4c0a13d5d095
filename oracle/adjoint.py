"""Derivative of lambda_1 with respect to the moments and to beta.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

What is differentiated.  lambda_1(k) = 1 / lambda_max(M) with M the top-left
k x k block of H_N^-1 (Sections 4.2 and 4.5).  The paper does not differentiate
it; the reading taken here is the first-order perturbation of a simple
eigenvalue of a symmetric matrix:

    d lambda_max = y^T dM y              (y the unit eigenvector of lambda_max),
    dM           = -E^T H^-1 dH H^-1 E   (E = the first k columns of I),

so that, with v = lambda_1 H^-1 E y,

    d lambda_1 = -d lambda_max / lambda_max^2 = v^T dH v.

H_N is a Hankel matrix, dH_ij = d mu_{i+j}, hence

    d lambda_1 / d mu_m = mubar_m = sum_{i+j=m} v_i v_j            (the adjoint)
    d lambda_1 / d beta = sum_m mubar_m d mu_m / d beta.

``grad`` evaluates these definitions directly in mpmath at a stated precision
(dense inverse, dense symmetric eigen-solver), for N up to a few dozen.

Parity status: pinned in tests/test_oracle_adjoint.py by (1) the eigenvalue
derivative of H_N itself when k = N (Hellmann-Feynman with the eigenvector of
H_N, a route that never forms H^-1), (2) central finite differences of the
forward lambda_1 along the moment tangent and along beta, (3) the closed form of
the smallest eigenvalue of a 2 x 2 Hankel matrix, and (4) the sensitivity of
those pins to planted mistakes.
"""
from dataclasses import dataclass
from typing import List, Sequence

import mpmath


def _mpf(x):
    """An input number (a Dyadic, an int or a Fraction) as an mpf; exact when the
    working precision holds its mantissa."""
    if hasattr(x, "M") and hasattr(x, "e"):
        return mpmath.ldexp(mpmath.mpf(x.M), x.e)
    if hasattr(x, "numerator"):
        return mpmath.mpf(x.numerator) / x.denominator
    return mpmath.mpf(x)


@dataclass
class Grad:
    lam1: object          # lambda_1(k) = 1 / lambda_max(M)
    y: List[object]       # unit eigenvector of M for lambda_max
    v: List[object]       # lambda_1 H^-1 E y
    mubar: List[object]   # d lambda_1 / d mu_m, m = 0 .. 2N-2
    dlam: object          # sum_m mubar_m dmu_m (None when dmu is not given)
    prec: int


def lambda1(mu: Sequence, N: int, k: int, prec: int):
    """lambda_1(k) alone (the forward map whose derivative ``grad`` gives)."""
    return grad(mu, None, N, k, prec).lam1


def grad(mu: Sequence, dmu, N: int, k: int, prec: int) -> Grad:
    """The definitions in the module header at ``prec`` bits.

    mu   moments mu_0 .. mu_{2N-2} (Dyadic, int or Fraction)
    dmu  d mu_m / d beta (same types), or None to skip the contraction
    """
    if not 1 <= k <= N:
        raise ValueError("need 1 <= k <= N")
    with mpmath.workprec(prec):
        m = [_mpf(mu[j]) for j in range(2 * N - 1)]
        H = mpmath.matrix(N, N)
        for i in range(N):
            for j in range(N):
                H[i, j] = m[i + j]
        Hi = mpmath.inverse(H)
        M = mpmath.matrix(k, k)
        for a in range(k):
            for b in range(k):
                M[a, b] = (Hi[a, b] + Hi[b, a]) / 2
        ev, Q = mpmath.eigsy(M)
        top = max(range(k), key=lambda j: ev[j])
        lam_max = ev[top]
        y = [Q[a, top] for a in range(k)]
        nrm = mpmath.sqrt(mpmath.fsum(t * t for t in y))
        y = [t / nrm for t in y]
        lam1 = 1 / lam_max
        # v = lambda_1 H^-1 E y: H^-1 E is the first k columns of H^-1
        v = [lam1 * mpmath.fsum(Hi[i, a] * y[a] for a in range(k)) for i in range(N)]
        mubar = []
        for s in range(2 * N - 1):
            lo, hi = max(0, s - (N - 1)), min(s, N - 1)
            mubar.append(mpmath.fsum(v[i] * v[s - i] for i in range(lo, hi + 1)))
        dlam = None
        if dmu is not None:
            dlam = mpmath.fsum(mubar[s] * _mpf(dmu[s]) for s in range(2 * N - 1))
        return Grad(lam1=lam1, y=y, v=v, mubar=mubar, dlam=dlam, prec=prec)
