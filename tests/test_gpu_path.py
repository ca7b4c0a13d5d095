"""GPU parity of the whole path: X (first k columns of L^-1) and the block of
H^-1 bit-exact with the oracle; lambda_1 and the truncation estimate within the
eigen-step's tolerance of the oracle's dense eigen-solve at doubled precision;
lambda_2 and lambda_3 (deflation) within the same tolerance scaled by
lambda_j / lambda_1."""
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


@pytest.mark.parametrize("beta,N,k,P,E,form", [
    (Fraction(1, 2), 64, 8, 2048, 16, "mfma"),
    (Fraction(1), 64, 8, 4096, 16, "valu"),
    (Fraction(1, 3), 40, 6, 1536, 1, "valu"),
    (Fraction(1, 2), 70, 20, 2176, 16, "mfma"),
    (Fraction(1, 3), 45, 32, 1024, 1, "mfma"),
])
def test_lambda_next_vs_oracle(beta, N, k, P, E, form):
    # The deflated block B - mu_1 y y^T / (y^T y) is formed at the eigen-step's
    # working precision (P + 96 bits relative to mu_1), and an eigenvector
    # error e moves the next eigenvalue by mu_1 e^2 only, so mu_j carries an
    # absolute error of about mu_1 2^-(P + 32) and lambda_j = 1 / mu_j a
    # relative one of (lambda_j / lambda_1) 2^-(P + 32); the bar is that with
    # the 96 bits of margin that lambda_1's test also keeps.
    say("next", beta, N, k, P, E, form)
    f, sv, bl, ev, fac, res = _run(beta, N, k, P, E, form)
    nxt = ctx().lambda_next(fac, 2)
    ref = C.eigen_next(bl, 2, P=P)
    with mpmath.workprec(2 * P + 64):
        prev = _mp(res["mant"], res["exp"])
        for g, r in zip(nxt, ref):
            assert g["j"] == r.j
            tol = mpmath.mpf(2) ** -(P - 64) * r.lam / ev.lam1
            lam = _mp(g["mant"], g["exp"])
            assert abs(lam / r.lam - 1) < tol, (r.j, lam, r.lam)
            lamk1 = _mp(g["mant_km1"], g["exp_km1"])
            assert abs(lamk1 / r.lam_km1 - 1) < tol * r.lam_km1 / r.lam
            assert abs(g["lambda"] / float(r.lam) - 1) < 1e-15
            assert g["trunc"] <= 0
            assert abs(g["trunc"] - float(r.trunc)) <= 1e-15 * abs(float(r.trunc)) + 3 * float(tol * r.lam_km1)
            assert lam > prev
            prev = lam
    # one eigenvalue only, and the shapes that cannot have an estimate
    one = ctx().lambda_next(fac, 1, want_mant=False)
    assert len(one) == 1 and one[0]["lambda"] == nxt[0]["lambda"]


def test_full_block_next_eigenvalues_n8():
    # k = N: lambda_2 and lambda_3 are the second and third eigenvalues of H_8,
    # isolated exactly from the characteristic polynomial
    N, P = 8, 1024
    say("next, k = N = 8")
    mu = moments(Fraction(1, 2), 2 * N - 1)
    fac = ctx().factor(mu, N, N, P, 1, "valu")
    ctx().lambda_min(fac)
    nxt = ctx().lambda_next(fac, 2)
    H = X.hankel([m.to_fraction() for m in mu], N)
    c = X.charpoly(H)
    tr = sum(H[i][i] for i in range(N))
    with mpmath.workprec(800):
        for g in nxt:
            root = X.kth_root(c, g["j"], tr, bits=400 + int(tr).bit_length())
            lam = _mp(g["mant"], g["exp"])
            assert abs(lam / (mpmath.mpf(root.numerator) / root.denominator) - 1) < mpmath.mpf(10) ** -90


def test_lambda_next_rejects_bad_count():
    from paper_1810_01478_amd import _lib as L
    mu = moments(Fraction(1, 2), 2 * 16 - 1)
    fac = ctx().factor(mu, 16, 3, 1024, 16, "valu")
    ctx().lambda_min(fac)
    ctx().lambda_next(fac, 1, want_mant=False)
    for bad in (0, 2, 3):
        with pytest.raises(L.HLError):
            ctx().lambda_next(fac, bad, want_mant=False)
