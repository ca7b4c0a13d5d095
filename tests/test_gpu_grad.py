"""GPU adjoint (hl_lambda_grad): d lambda_1 / d beta against the oracle's
definition at small N (at least 30 digits), against central differences of the
GPU's own lambda_1 along the moment tangent at the differentiation workload's
sizes (beta in {0.45, 0.5, 0.55}, N in {128, 256, 512}, P = 16384), and through
the torch.autograd.Function."""
import functools
import json
import os
from fractions import Fraction

import mpmath
import pytest
import torch

from hankel_inputs import Dyadic, dmoments_dbeta, moments
from oracle import adjoint as A

from gpu_util import ctx, say

pytestmark = pytest.mark.gpu


def _mp(mant, exp):
    return mpmath.ldexp(mpmath.mpf(mant), exp)


def _lam_mp(res):
    return _mp(res["mant"], res["exp"])


def _grad_mp(res, g):
    # d lambda_1 = lambda_1^2 num 2^num_shift / den, all exact integers from the GPU
    lam = _lam_mp(res)
    return lam * lam * mpmath.ldexp(mpmath.mpf(g["num"]), g["num_shift"]) / g["den"]


def _run(mu, dmu, N, k, P, E, form):
    fac = ctx().factor(mu, N, k, P, E, form)
    res = ctx().lambda_min(fac)
    g = ctx().lambda_grad(fac, dmu)
    return fac, res, g


def _along(mu, dmu, h_exp):
    """mu + 2^h_exp dmu as exact dyadics."""
    out = []
    for a, d in zip(mu, dmu):
        e0 = min(a.e, d.e + h_exp)
        out.append(Dyadic((a.M << (a.e - e0)) + (d.M << (d.e + h_exp - e0)), e0))
    return out


@pytest.mark.parametrize("beta,N,k,P,E,form", [
    (Fraction(1, 2), 24, 6, 2048, 16, "valu"),
    (Fraction(9, 20), 20, 5, 1536, 7, "mfma"),
    (Fraction(1, 2), 40, 8, 4096, 16, "mfma"),
    (Fraction(1), 33, 1, 1024, 16, "valu"),
    (Fraction(11, 20), 16, 16, 2048, 16, "mfma"),
])
def test_grad_vs_oracle(beta, N, k, P, E, form):
    say("grad vs oracle", beta, N, k, P, E, form)
    mu = moments(beta, 2 * N - 1, P + 64)
    dmu = dmoments_dbeta(beta, 2 * N - 1, P + 64)
    fac, res, g = _run(mu, dmu, N, k, P, E, form)
    o = A.grad(mu, dmu, N, k, 3 * P)
    with mpmath.workprec(3 * P):
        gd = _grad_mp(res, g)
        rel = abs(gd / o.dlam - 1)
        say("  digits", mpmath.nstr(-mpmath.log10(rel) if rel else mpmath.inf, 5))
        assert rel < mpmath.mpf(10) ** -30
        assert abs(g["dlambda1"] / float(o.dlam) - 1) < 1e-14
        assert abs(g["lambda1"] / float(o.lam1) - 1) < 1e-14


@functools.lru_cache(maxsize=8)
def _inputs(beta, count, bits):
    """Moments and their beta-derivatives rounded to `bits` bits (Gamma at
    rational points to 16 kbit is slow on the host: computed once per test
    session)."""
    return moments(beta, count, bits), dmoments_dbeta(beta, count, bits)


def _central_difference_case(beta, N, k, P, E, form):
    say("grad vs central difference", beta, N, k, P, E, form)
    mu, dmu = _inputs(beta, 2 * N - 1, P + 64)
    fac, res, g = _run(mu, dmu, N, k, P, E, form)
    h_exp = -100  # h = 2^-100 ~ 7.9e-31
    lp = ctx().lambda_min(ctx().factor(_along(mu, dmu, h_exp), N, k, P, E, form))
    neg = [Dyadic(-d.M, d.e) for d in dmu]
    lm = ctx().lambda_min(ctx().factor(_along(mu, neg, h_exp), N, k, P, E, form))
    with mpmath.workprec(2 * P):
        fd = (_lam_mp(lp) - _lam_mp(lm)) / mpmath.ldexp(1, h_exp + 1)
        gd = _grad_mp(res, g)
        rel = abs(gd / fd - 1)
        say("  d lambda_1 / d beta", mpmath.nstr(gd, 25), "digits vs difference",
            mpmath.nstr(-mpmath.log10(rel) if rel else mpmath.inf, 5))
        assert rel < mpmath.mpf(10) ** -40
        assert abs(g["dlambda1"] / float(gd) - 1) < 1e-14


@pytest.mark.parametrize("N", [128, 256, 512])
def test_grad_central_difference_half(N):
    _central_difference_case(Fraction(1, 2), N, 8, 16384, 16, "mfma")


@pytest.mark.timeout(600)
@pytest.mark.parametrize("beta", [Fraction(9, 20), Fraction(11, 20)])
def test_grad_central_difference_off_half(beta):
    # moments of beta = p/q need Gamma at p rational points to 16 kbit (slow on
    # the host); one N per beta
    _central_difference_case(beta, 128, 8, 16384, 16, "mfma")


def _records(N):
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                        "oracle_adjoint_n%d_p16384.json" % N)
    if not os.path.exists(path):
        return []
    with open(path) as f:
        return json.load(f)["records"]


@pytest.mark.timeout(900)
@pytest.mark.parametrize("N", [128, 256])
def test_grad_vs_oracle_records_at_differentiation_sizes(N):
    """d lambda_1 / d beta at beta in {9/20, 1/2, 11/20}, P = 16384, k = 8
    against the oracle's definition evaluated offline at 8192 bits
    (tests/golden/make_adjoint_goldens.py); the records keep 100 digits."""
    recs = _records(N)
    if not recs:
        pytest.skip("oracle record for N = %d not written yet" % N)
    for rec in recs:
        num, den = (int(x) for x in rec["beta"].split("/"))
        beta = Fraction(num, den)
        k, P, E = rec["k"], rec["P"], rec["E"]
        say("grad vs oracle record", beta, N, k, P, E)
        mu, dmu = _inputs(beta, 2 * N - 1, rec["inputs_rounded_to_bits"])
        fac, res, g = _run(mu, dmu, N, k, P, E, "mfma")
        with mpmath.workprec(2 * P):
            gd = _grad_mp(res, g)
            ref = mpmath.mpf(rec["dlam1_dbeta"])
            rel = abs(gd / ref - 1)
            rl = abs(_lam_mp(res) / mpmath.mpf(rec["lam1"]) - 1)
            d1 = -mpmath.log10(rel) if rel else mpmath.inf
            d2 = -mpmath.log10(rl) if rl else mpmath.inf
            say("  d lambda_1 / d beta digits", mpmath.nstr(d1, 5), "lambda_1 digits", mpmath.nstr(d2, 5))
            assert rel < mpmath.mpf(10) ** -90 and rl < mpmath.mpf(10) ** -90
        del fac


def test_autograd_function():
    from paper_1810_01478_amd.api import lambda1
    N, k, P = 32, 8, 2048
    say("autograd", N, k, P)
    beta = torch.tensor(0.45, dtype=torch.float64, requires_grad=True)
    lam = lambda1(beta, N, k, P, context=ctx())
    lam.backward()
    b = Fraction(9, 20)
    mu = moments(b, 2 * N - 1, P + 64)
    dmu = dmoments_dbeta(b, 2 * N - 1, P + 64)
    o = A.grad(mu, dmu, N, k, 3 * P)
    assert abs(lam.item() / float(o.lam1) - 1) < 1e-14
    assert abs(float(beta.grad) / float(o.dlam) - 1) < 1e-14
