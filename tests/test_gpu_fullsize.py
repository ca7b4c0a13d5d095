"""Parity at the benchmark workload itself (beta = 1/2, N = 1024, k = 16,
P = 49152, E = 16), in the launch configuration bench.py times (default
Schur-update form: three Karatsuba levels, pivot lookahead).  The oracle cannot
factor the whole matrix in test time, so the checks are on what it can compute
and on properties that hold at any size:
  * sampled outputs: the pivots, balance exponents and multipliers of the
    leading 48 columns equal the oracle's factorisation of the leading 48 x 48
    block (the leading block of an LDL^T is the LDL^T of the leading block, and
    the exponent blocks of 16 rows coincide), bit for bit;
  * the first 64 columns, factored with the plain int8 digit-product update,
    give the same pivots, multipliers and live trailing matrix as the default
    form at full size;
  * lambda_1 does not depend on the precision: at P = 49152 and at 12288 bits
    it agrees to far more digits than a double holds (the paper validates its
    precision the same way), and the truncation estimate is <= 0 (interlacing)."""
from fractions import Fraction

import mpmath
import pytest

from hankel_inputs import moments
from oracle import contract as C

from gpu_util import ctx, say

pytestmark = pytest.mark.gpu

BETA, N, K, P, E = Fraction(1, 2), 1024, 16, 49152, 16


def test_full_size_leading_block_and_precision_agreement():
    import torch
    c = ctx()
    mu = moments(BETA, 2 * N - 1)
    say("full size factor", N, P)
    fac = c.factor(mu, N, K, P, E, "mfma")
    res = c.lambda_min(fac)
    assert res["trunc"] <= 0.0
    say("  lambda1", res["lambda1"], "trunc", res["trunc"])
    # sampled outputs against the oracle: the leading 48 x 48 block
    Ns = 48
    f = C.factor(mu, Ns, P, E)
    assert fac.pivots()[:Ns] == f.d
    assert fac.h_list()[:Ns] == f.h
    for i in range(Ns - 1):
        assert fac.multipliers(i, range(i + 1, Ns)) == [f.b[i][r] for r in range(i + 1, Ns)], i
    # the same lambda_1 at 12288 bits
    P2 = 12288
    fac2 = c.factor(mu, N, K, P2, E, "mfma")
    res2 = c.lambda_min(fac2)
    with mpmath.workprec(4 * P2):
        a = mpmath.ldexp(mpmath.mpf(res["mant"]), res["exp"])
        b = mpmath.ldexp(mpmath.mpf(res2["mant"]), res2["exp"])
        rel = abs(a / b - 1)
        lg = float(mpmath.log10(rel)) if rel else float("-inf")
        say("  lambda1 P vs 12288 bits: log10 relative difference %.1f" % lg)
        assert rel < mpmath.mpf(10) ** -200
    del fac2
    torch.cuda.empty_cache()


def test_full_size_first_panels_equal_digit_product():
    import torch
    c = ctx()
    mu = moments(BETA, 2 * N - 1)
    cols = 64
    say("full size first", cols, "columns: default vs digit product")
    try:
        c.set_karatsuba(-1)
        fa = c.factor_cols(mu, N, K, P, E, "mfma", 0, cols)
        c.sync(fa)
        c.set_karatsuba(0)
        fb = c.factor_cols(mu, N, K, P, E, "mfma", 0, cols)
        c.sync(fb)
    finally:
        c.set_karatsuba(-1)
    nl = P // 32
    assert torch.equal(fa.d[:cols * 2 * nl], fb.d[:cols * 2 * nl])
    assert torch.equal(fa.l, fb.l)
    so, tb = fa.sizes.trail_offset, 1024 * 2 * nl * 4
    for R in range(cols // 32, N // 32):
        t0 = so + (R * (R + 1) // 2 + cols // 32) * tb
        t1 = so + (R * (R + 1) // 2 + R + 1) * tb
        assert torch.equal(fa.ws[t0:t1], fb.ws[t0:t1]), R
