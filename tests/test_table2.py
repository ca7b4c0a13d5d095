"""The paper's Table 2 (beta = 1/2, k = 8) as golden values.

CPU: the fixture reads back whole and keeps the orderings the mathematics fixes
(lambda_1 < lambda_2 < lambda_3, each decreasing in N; truncation estimates
negative, by Cauchy interlacing of the k-1 block inside the k block).
GPU: the whole path (moments -> LDL^T -> first k columns of L^-1 -> block of
H^-1 -> eigen-step) at N = 500 and N = 1000, k = 8, reproduces the printed
lambda_1 to the 16 printed digits and the truncation estimate within the
double-precision error of the paper's own difference, and lambda_2, lambda_3
with their estimates within the error of the paper's double-precision
eigen-solve (golden_table2.paper_error).  The same at N = 1500 .. 2500 through
the paper's precision scan (paper_1810_01478_amd.table2, E = 1), started at the
precision Table 2 quotes."""
from fractions import Fraction

import pytest

from golden_table2 import paper_error, table2


def test_fixture_orderings():
    t = table2()
    assert sorted(t) == [500, 1000, 1500, 2000, 2500, 3000, 3500, 4000, 4500]
    prev = None
    for N in sorted(t):
        r = t[N]
        assert 0 < r.lambda1 < r.lambda2 < r.lambda3
        assert r.trunc1 < 0 and r.trunc2 < 0 and r.trunc3 < 0
        if prev is not None:
            assert r.lambda1 < prev.lambda1 and r.lambda2 < prev.lambda2 and r.lambda3 < prev.lambda3
        prev = r


def test_scan_agreement_rule():
    # host logic of the precision scan: a failed run agrees with nothing, and
    # every eigenvalue of both blocks must agree to the relative tolerance
    from paper_1810_01478_amd.table2 import agree
    a = {"lambda": [0.1, 1.0, 30.0], "lambda_km1": [0.1, 1.0, 30.0]}
    b = {"lambda": [0.1 * (1 + 5e-16), 1.0, 30.0], "lambda_km1": [0.1, 1.0, 30.0]}
    c = {"lambda": [0.1, 1.0, 30.0], "lambda_km1": [0.1, 1.0, 30.0 * (1 + 4e-15)]}
    assert agree(a, b, 1e-15)
    assert not agree(a, c, 1e-15)
    assert not agree(a, {"error": "HL_ENOTPD"}, 1e-15)
    assert not agree({"error": "HL_ENOTPD"}, {"error": "HL_ENOTPD"}, 1e-15)


@pytest.mark.gpu
@pytest.mark.parametrize("N", [500, 1000])
def test_lambda1_reproduces_table2(N):
    from hankel_inputs import moments
    from hankel_inputs.moments import precision_rule
    from gpu_util import ctx, say
    row = table2()[N]
    beta = Fraction(1, 2)
    P = precision_rule(beta, N)
    say("table 2", N, P)
    mu = moments(beta, 2 * N - 1, P + 64)
    fac = ctx().factor(mu, N, 8, P, 16, "mfma")
    res = ctx().lambda_min(fac)
    say("  lambda1", repr(res["lambda1"]), "paper", row.lambda1, "trunc", res["trunc"], "paper", row.trunc1)
    # 16 printed digits, computed there in double precision from the block
    assert abs(res["lambda1"] / row.lambda1 - 1) < 2e-15
    # the paper's estimate is the difference of two eigenvalues computed in
    # double precision, each good to about the 2e-15 relative agreement above,
    # so it carries an absolute error of that order (here it is exact)
    assert res["trunc"] < 0
    assert abs(res["trunc"] - row.trunc1) <= 2e-15 * row.lambda1
    for g in ctx().lambda_next(fac, 2, want_mant=False):
        e_lam, e_tr = paper_error(row, g["j"])
        lam_p = (row.lambda2, row.lambda3)[g["j"] - 2]
        tr_p = (row.trunc2, row.trunc3)[g["j"] - 2]
        say("  lambda%d" % g["j"], repr(g["lambda"]), "paper", lam_p, "trunc", g["trunc"], "paper", tr_p)
        assert abs(g["lambda"] - lam_p) <= e_lam
        assert g["trunc"] < 0
        assert abs(g["trunc"] - tr_p) <= e_tr


@pytest.mark.gpu
@pytest.mark.parametrize("N", [1500, 2000, 2500])
def test_precision_scan_reproduces_table2(N):
    from paper_1810_01478_amd import table2 as T
    from gpu_util import ctx, say
    row = table2()[N]
    say("table 2 scan", N, "from", row.K_bits)
    res = T.precision_scan(ctx(), Fraction(1, 2), N, k=8, count=2, P_start=row.K_bits, step=1024)
    P = res["required_P"]
    got = res["row"]
    say("  required P", P, "lambda", got["lambda"], "trunc", got["trunc"])
    # the scan's rule: P and P + 1024 agree to 1e-15, and P - 1024 (if it was
    # run) did not agree with P
    assert T.agree(got, res["check"], 1e-15)
    if P > row.K_bits:
        below = [r for r in res["runs"] if r["P"] == P - 1024][0]
        assert not T.agree(below, got, 1e-15)
    assert abs(got["lambda"][0] / row.lambda1 - 1) < 2e-15
    assert got["trunc"][0] < 0 and abs(got["trunc"][0] - row.trunc1) <= 2e-15 * row.lambda1
    for j in (2, 3):
        e_lam, e_tr = paper_error(row, j)
        assert abs(got["lambda"][j - 1] - (row.lambda2, row.lambda3)[j - 2]) <= e_lam
        assert got["trunc"][j - 1] < 0
        assert abs(got["trunc"][j - 1] - (row.trunc2, row.trunc3)[j - 2]) <= e_tr
