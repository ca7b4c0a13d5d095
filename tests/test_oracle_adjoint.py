"""Pins of the oracle's derivative of lambda_1 (oracle/adjoint.py) and of the
moment derivative generator: nothing here reuses the formula being checked."""
from fractions import Fraction

import mpmath
import pytest

from hankel_inputs import dmoments_dbeta, moments
from oracle import adjoint as A


def _mp(x):
    return A._mpf(x)


def _central_difference_along(mu, dmu, N, k, prec, h):
    """(lambda_1(mu + h dmu) - lambda_1(mu - h dmu)) / 2h, forward map only."""
    with mpmath.workprec(prec):
        hp = mpmath.mpf(h)
        up = [_mp(mu[j]) + hp * _mp(dmu[j]) for j in range(2 * N - 1)]
        dn = [_mp(mu[j]) - hp * _mp(dmu[j]) for j in range(2 * N - 1)]
        return (A.lambda1(up, N, k, prec) - A.lambda1(dn, N, k, prec)) / (2 * hp)


def test_k_equals_n_is_the_eigenvalue_derivative_of_h():
    # k = N: lambda_1(N) is the smallest eigenvalue of H_N itself, and its
    # derivative is phi^T H' phi with phi the unit eigenvector of H_N (no H^-1)
    N, prec = 8, 600
    beta = Fraction(1, 2)
    mu = moments(beta, 2 * N - 1)
    dmu = dmoments_dbeta(beta, 2 * N - 1, prec + 64)
    g = A.grad(mu, dmu, N, N, prec)
    with mpmath.workprec(prec):
        H = mpmath.matrix(N, N)
        for i in range(N):
            for j in range(N):
                H[i, j] = _mp(mu[i + j])
        ev, Q = mpmath.eigsy(H)
        j0 = min(range(N), key=lambda j: ev[j])
        phi = [Q[i, j0] for i in range(N)]
        hf = mpmath.fsum(phi[i] * phi[j] * _mp(dmu[i + j]) for i in range(N) for j in range(N))
        assert abs(g.lam1 / ev[j0] - 1) < mpmath.mpf(2) ** -(prec - 200)
        assert abs(g.dlam / hf - 1) < mpmath.mpf(2) ** -(prec - 250)


@pytest.mark.parametrize("beta,N,k", [(Fraction(1, 2), 10, 4), (Fraction(9, 20), 8, 3),
                                      (Fraction(1), 9, 9), (Fraction(1, 3), 7, 1)])
def test_central_difference_along_the_moment_tangent(beta, N, k):
    prec = 900
    mu = moments(beta, 2 * N - 1, prec + 64)
    dmu = dmoments_dbeta(beta, 2 * N - 1, prec + 64)
    g = A.grad(mu, dmu, N, k, prec)
    fd = _central_difference_along(mu, dmu, N, k, prec, mpmath.ldexp(1, -80))
    with mpmath.workprec(prec):
        assert abs(fd / g.dlam - 1) < mpmath.mpf(10) ** -40


def test_central_difference_in_beta():
    # moments recomputed at beta +- h: also checks the moment derivative generator
    N, k, prec = 6, 3, 500
    beta, h = Fraction(1, 2), Fraction(1, 10**20)
    dmu = dmoments_dbeta(beta, 2 * N - 1, prec + 64)
    g = A.grad(moments(beta, 2 * N - 1), dmu, N, k, prec)
    lp = A.lambda1(moments(beta + h, 2 * N - 1, prec + 64), N, k, prec)
    lm = A.lambda1(moments(beta - h, 2 * N - 1, prec + 64), N, k, prec)
    with mpmath.workprec(prec):
        fd = (lp - lm) / (2 * _mp(h))
        assert abs(fd / g.dlam - 1) < mpmath.mpf(10) ** -30


def test_two_by_two_closed_forms():
    # N = 2: lambda_min = (a + c)/2 - sqrt(((a - c)/2)^2 + b^2) with a, b, c =
    # mu_0, mu_1, mu_2; for k = 1, lambda_1 = 1 / (H^-1)_00 = (a c - b^2) / c
    prec = 400
    beta = Fraction(9, 20)
    mu = moments(beta, 3, prec + 64)
    dmu = dmoments_dbeta(beta, 3, prec + 64)
    with mpmath.workprec(prec):
        a, b, c = (_mp(t) for t in mu)
        da, db, dc = (_mp(t) for t in dmu)
        root = mpmath.sqrt(((a - c) / 2) ** 2 + b * b)
        lam = (a + c) / 2 - root
        dlam = (da + dc) / 2 - ((a - c) * (da - dc) / 4 + b * db) / root
        g2 = A.grad(mu, dmu, 2, 2, prec)
        assert abs(g2.lam1 / lam - 1) < mpmath.mpf(2) ** -(prec - 40)
        assert abs(g2.dlam / dlam - 1) < mpmath.mpf(2) ** -(prec - 60)
        l1 = (a * c - b * b) / c
        dl1 = ((da * c + a * dc - 2 * b * db) * c - (a * c - b * b) * dc) / (c * c)
        g1 = A.grad(mu, dmu, 2, 1, prec)
        assert abs(g1.lam1 / l1 - 1) < mpmath.mpf(2) ** -(prec - 40)
        assert abs(g1.dlam / dl1 - 1) < mpmath.mpf(2) ** -(prec - 60)


def test_planted_mistakes_are_caught():
    # plausible slips in the adjoint, made from the oracle's own outputs, all
    # fail the central-difference pin
    N, k, prec = 9, 4, 900
    beta = Fraction(1, 2)
    mu = moments(beta, 2 * N - 1)
    dmu = dmoments_dbeta(beta, 2 * N - 1, prec + 64)
    g = A.grad(mu, dmu, N, k, prec)
    fd = _central_difference_along(mu, dmu, N, k, prec, mpmath.ldexp(1, -80))
    with mpmath.workprec(prec):
        tol = mpmath.mpf(10) ** -40
        assert abs(fd / g.dlam - 1) < tol
        # v without the factor lambda_1
        assert abs(fd / (g.dlam / g.lam1 ** 2) - 1) > tol
        # adjoint contracted with the neighbouring moment derivative
        shifted = mpmath.fsum(g.mubar[s] * _mp(dmu[s + 1]) for s in range(2 * N - 2))
        assert abs(fd / shifted - 1) > tol
        # mubar with each unordered pair counted once
        once = []
        for s in range(2 * N - 1):
            lo, hi = max(0, s - (N - 1)), min(s, N - 1)
            once.append(mpmath.fsum(g.v[i] * g.v[s - i] for i in range(lo, hi + 1) if i <= s - i))
        wrong = mpmath.fsum(once[s] * _mp(dmu[s]) for s in range(2 * N - 1))
        assert abs(fd / wrong - 1) > tol
        # y taken at the other end of the block's spectrum
        H = mpmath.matrix(N, N)
        for i in range(N):
            for j in range(N):
                H[i, j] = _mp(mu[i + j])
        Hi = mpmath.inverse(H)
        M = mpmath.matrix(k, k)
        for a in range(k):
            for b in range(k):
                M[a, b] = Hi[a, b]
        ev, Q = mpmath.eigsy(M)
        low = min(range(k), key=lambda j: ev[j])
        v = [g.lam1 * mpmath.fsum(Hi[i, a] * Q[a, low] for a in range(k)) for i in range(N)]
        wrong = mpmath.fsum(v[i] * v[j] * _mp(dmu[i + j]) for i in range(N) for j in range(N))
        assert abs(fd / wrong - 1) > tol


@pytest.mark.parametrize("beta", [Fraction(9, 20), Fraction(1, 2), Fraction(11, 20), Fraction(1, 3), Fraction(1)])
def test_moment_derivative_against_numerical_differentiation(beta):
    # d/d beta of Gamma((m+1)/beta)/beta by mpmath's numerical differentiation
    bits = 300
    dmu = dmoments_dbeta(beta, 12, bits)
    with mpmath.workprec(bits + 200):
        b0 = mpmath.mpf(beta.numerator) / beta.denominator
        for m in (0, 1, 4, 11):
            d = mpmath.diff(lambda b: mpmath.gamma((m + 1) / b) / b, b0)
            assert abs(_mp(dmu[m]) / d - 1) < mpmath.mpf(10) ** -60
