"""Exact rational arithmetic for tiny N.  TEST INFRASTRUCTURE ONLY.

These functions are the plain definitions, with no rounding at all:

* ``ldl``: H = L D L^T over the rationals (Section 4.3, Algorithm 1 in exact
  arithmetic; no pivoting, footnote of Section 4.3);
* ``linv_cols``: the first m columns of L^-1 (Algorithm 4 in exact arithmetic);
* ``hinv_block``: eq. ``equ:index`` summed exactly over l;
* ``charpoly``: the characteristic polynomial of H_N, by the Faddeev-LeVerrier
  recurrence in rationals, and ``smallest_root`` which isolates its smallest
  root by bisection on exact sign changes (the brute-force smallest eigenvalue);
  ``kth_root`` the same for the j-th smallest root (lambda_2, lambda_3).

Parity status: pinned by closed forms (beta = 1: D_m = (m!)^2, L_ij = C(i,j) i!/j!,
det H_N = prod (m!)^2), by H == L D L^T exactly, and by sympy's independent
characteristic polynomial in tests/test_oracle_pins.py; ``kth_root`` by a
polynomial with known rational roots in tests/test_oracle_pins.py.
"""

from __future__ import annotations

from fractions import Fraction
from typing import List, Sequence, Tuple


def hankel(mu: Sequence[Fraction], N: int) -> List[List[Fraction]]:
    """Section 2, eq. ``matrix``: H_N = (mu_{i+j}), i, j = 0..N-1."""
    return [[Fraction(mu[i + j]) for j in range(N)] for i in range(N)]


def ldl(H: List[List[Fraction]]) -> Tuple[List[List[Fraction]], List[Fraction]]:
    """Exact LDL^T by Algorithm 1: for each column i, B_i = A_i / A_i[i], then
    A_j[k] -= A_i[j] B_i[k] for k >= j > i."""
    N = len(H)
    A = [[Fraction(H[r][c]) for c in range(N)] for r in range(N)]
    L = [[Fraction(int(r == c)) for c in range(N)] for r in range(N)]
    D = []
    for i in range(N):
        di = A[i][i]
        if di == 0:
            raise ZeroDivisionError("singular leading block at %d" % i)
        D.append(di)
        for r in range(i + 1, N):
            L[r][i] = A[r][i] / di
        for c in range(i + 1, N):
            for r in range(c, N):
                A[r][c] -= A[c][i] * L[r][i]
    return L, D


def linv_cols(L: List[List[Fraction]], m: int) -> List[List[Fraction]]:
    """Algorithm 4: the first m columns of L^-1 (unit lower triangular L), by
    forward substitution row by row; column a of the result solves L x = e_a."""
    N = len(L)
    X = [[Fraction(0)] * m for _ in range(N)]
    for a in range(m):
        X[a][a] = Fraction(1)
        for r in range(a + 1, N):
            X[r][a] = -sum((L[r][i] * X[i][a] for i in range(a, r)), Fraction(0))
    return X


def hinv_block(X: List[List[Fraction]], D: List[Fraction], k: int) -> List[List[Fraction]]:
    """eq. ``equ:index``: (H^-1)_ab = sum_l (L^-1)_la (L^-1)_lb / D_ll."""
    N = len(D)
    return [[sum((X[l][a] * X[l][b] / D[l] for l in range(N)), Fraction(0))
             for b in range(k)] for a in range(k)]


def charpoly(H: List[List[Fraction]]) -> List[Fraction]:
    """Coefficients c_0..c_N of det(x I - H) = sum c_j x^j, by Faddeev-LeVerrier:
    M_1 = I, c_{N-1} = -tr H; M_k = H M_{k-1} + c_{N-k+1} I,
    c_{N-k} = -tr(H M_k) / k."""
    N = len(H)
    c = [Fraction(0)] * (N + 1)
    c[N] = Fraction(1)
    M = [[Fraction(int(i == j)) for j in range(N)] for i in range(N)]
    for kk in range(1, N + 1):
        if kk > 1:
            HM = [[sum((H[i][l] * M[l][j] for l in range(N)), Fraction(0)) for j in range(N)]
                  for i in range(N)]
            M = [[HM[i][j] + (c[N - kk + 1] if i == j else 0) for j in range(N)] for i in range(N)]
        HM = [[sum((H[i][l] * M[l][j] for l in range(N)), Fraction(0)) for j in range(N)]
              for i in range(N)]
        c[N - kk] = -sum((HM[i][i] for i in range(N)), Fraction(0)) / kk
    return c


def _peval(c: List[Fraction], x: Fraction) -> Fraction:
    v = Fraction(0)
    for coef in reversed(c):
        v = v * x + coef
    return v


def _prem(a: List[Fraction], b: List[Fraction]) -> List[Fraction]:
    """Remainder of a / b (coefficient lists, lowest degree first)."""
    a = list(a)
    while len(b) and b[-1] == 0:
        b = b[:-1]
    while len(a) >= len(b) and any(a):
        if a[-1] == 0:
            a.pop()
            continue
        q = a[-1] / b[-1]
        sh = len(a) - len(b)
        for j in range(len(b)):
            a[sh + j] -= q * b[j]
        a.pop()
    while a and a[-1] == 0:
        a.pop()
    return a


def sturm_chain(c: List[Fraction]) -> List[List[Fraction]]:
    """p, p', and p_{k+1} = -rem(p_{k-1}, p_k) until the remainder vanishes."""
    p0 = list(c)
    p1 = [j * c[j] for j in range(1, len(c))]
    chain = [p0, p1]
    while True:
        r = _prem(chain[-2], chain[-1])
        if not r:
            return chain
        chain.append([-v for v in r])


def _sign_changes(chain, x: Fraction) -> int:
    signs = [s for s in (_peval(p, x) for p in chain) if s != 0]
    return sum(1 for u, v in zip(signs, signs[1:]) if (u > 0) != (v > 0))


def smallest_root(c: List[Fraction], hi: Fraction, bits: int = 200) -> Fraction:
    """Smallest positive root of a polynomial with real roots (the characteristic
    polynomial of a positive definite matrix): Sturm's theorem counts the roots
    in (0, x], and the bracket [0, hi] is halved ``bits`` times keeping at least
    one root on the left."""
    chain = sturm_chain(c)
    v0 = _sign_changes(chain, Fraction(0))
    lo, up = Fraction(0), Fraction(hi)
    if v0 - _sign_changes(chain, up) < 1:
        raise ValueError("no root below hi")
    for _ in range(bits):
        mid = (lo + up) / 2
        if v0 - _sign_changes(chain, mid) >= 1:
            up = mid
        else:
            lo = mid
    return (lo + up) / 2


def kth_root(c: List[Fraction], j: int, hi: Fraction, bits: int = 200) -> Fraction:
    """j-th smallest positive root of a polynomial whose roots are real and
    simple (the characteristic polynomial of a positive definite matrix with
    distinct eigenvalues): Sturm's theorem counts the roots in (0, x], and the
    bracket [0, hi] is halved ``bits`` times keeping at least j roots in (0, up]
    and fewer than j in (0, lo]."""
    chain = sturm_chain(c)
    v0 = _sign_changes(chain, Fraction(0))
    lo, up = Fraction(0), Fraction(hi)
    if v0 - _sign_changes(chain, up) < j:
        raise ValueError("fewer than %d roots below hi" % j)
    for _ in range(bits):
        mid = (lo + up) / 2
        if v0 - _sign_changes(chain, mid) >= j:
            up = mid
        else:
            lo = mid
    return (lo + up) / 2
