"""GPU parity of the whole path: X (first k columns of L^-1) and the block of
H^-1 bit-exact with the oracle; lambda_1 and the truncation estimate within the
eigen-step's tolerance of the oracle's dense eigen-solve at doubled precision."""
from fractions import Fraction

import mpmath
import pytest

from hankel_inputs import moments
from oracle import contract as C
from oracle import exact as X

from gpu_util import ctx, say

pytestmark = pytest.mark.gpu


def _mp(mant, exp):
    return mpmath.ldexp(mpmath.mpf(mant), exp)


def _run(beta, N, k, P, E, form):
    mu = moments(beta, 2 * N - 1)
    f, sv, bl, ev = C.lambda_min(mu, N, k, P, E)
    fac = ctx().factor(mu, N, k, P, E, form)
    res = ctx().lambda_min(fac)
    return f, sv, bl, ev, fac, res


@pytest.mark.parametrize("beta,N,k,P,E,form", [
    (Fraction(1, 2), 64, 8, 2048, 16, "valu"),
    (Fraction(1, 2), 80, 5, 1024, 7, "valu"),
    (Fraction(1), 64, 8, 4096, 16, "valu"),
    (Fraction(1, 3), 40, 6, 1536, 1, "valu"),
    (Fraction(1, 2), 64, 8, 2048, 16, "mfma"),
    (Fraction(1, 2), 70, 20, 2176, 16, "mfma"),   # k > 16 columns, a partial second limb range
    (Fraction(1, 3), 45, 32, 1024, 1, "mfma"),    # k = 32, the widest target
])
def test_block_and_lambda_vs_oracle(beta, N, k, P, E, form):
    say("path", beta, N, k, P, E, form)
    f, sv, bl, ev, fac, res = _run(beta, N, k, P, E, form)
    Xg = fac.linv()
    for r in range(N):
        assert Xg[r] == sv.X[r], r
    blk, bexp = fac.block()
    assert bexp == bl.blk_exp
    assert blk == bl.blk
    with mpmath.workprec(2 * P + 64):
        lam = _mp(res["mant"], res["exp"])
        assert abs(lam / ev.lam1 - 1) < mpmath.mpf(2) ** -(P - 64), (lam, ev.lam1)
        lamk1 = _mp(res["mant_km1"], res["exp_km1"])
        assert abs(lamk1 / ev.lam1_km1 - 1) < mpmath.mpf(2) ** -(P - 64)
        assert abs(res["lambda1"] / float(ev.lam1) - 1) < 1e-15
        assert res["trunc"] <= 0
        assert abs(res["trunc"] - float(ev.trunc)) <= 1e-12 * abs(float(ev.trunc)) + 1e-300


def test_full_block_equals_smallest_eigenvalue_n8():
    # k = N: the block is all of H^-1, so lambda_1 is the smallest eigenvalue,
    # isolated exactly from the characteristic polynomial
    N, P = 8, 1024
    say("k = N = 8")
    mu = moments(Fraction(1, 2), 2 * N - 1)
    fac = ctx().factor(mu, N, N, P, 1, "valu")
    res = ctx().lambda_min(fac)
    H = X.hankel([m.to_fraction() for m in mu], N)
    c = X.charpoly(H)
    tr = sum(H[i][i] for i in range(N))
    root = X.smallest_root(c, tr, bits=400 + int(tr).bit_length())
    with mpmath.workprec(800):
        lam = _mp(res["mant"], res["exp"])
        assert abs(lam / (mpmath.mpf(root.numerator) / root.denominator) - 1) < mpmath.mpf(10) ** -100
