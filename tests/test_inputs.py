"""Pins of the moment generator (Section 2, eq. ``moments``)."""
import math
from fractions import Fraction

import mpmath
import pytest

from hankel_inputs import moments, dmoments_dbeta, pack_limbs, unpack_limbs, batch_configs, precision_rule


def test_beta_one_is_factorial():
    mu = moments(1, 40)
    assert [m.M for m in mu] == [math.factorial(j) for j in range(40)]
    assert all(m.e == 0 for m in mu)


def test_beta_half_is_2_odd_factorial():
    mu = moments(Fraction(1, 2), 40)
    assert [m.M for m in mu] == [2 * math.factorial(2 * j + 1) for j in range(40)]


def test_beta_third():
    mu = moments(Fraction(1, 3), 30)
    assert [m.M for m in mu] == [3 * math.factorial(3 * j + 2) for j in range(30)]


@pytest.mark.parametrize("beta", [Fraction(2, 3), Fraction(9, 20), Fraction(11, 20)])
def test_irrational_moments_match_gamma(beta):
    # independent route: mpmath.gamma evaluated directly at each argument
    mu = moments(beta, 25, mant_bits=256)
    with mpmath.workprec(400):
        for j, m in enumerate(mu):
            ref = mpmath.gamma(mpmath.mpf(beta.denominator * (j + 1)) / beta.numerator) / (mpmath.mpf(beta.numerator) / beta.denominator)
            val = mpmath.ldexp(mpmath.mpf(m.M), m.e)
            assert abs(val / ref - 1) < mpmath.mpf(2) ** -250
            assert abs(m.M).bit_length() == 256 or m.e >= -1


def test_half_integer_gamma_route_exact_parts():
    # beta = 2/3: mu_1 = (3/2) Gamma(3) = 3 exactly; mu_0 = (3/2) Gamma(3/2) = (3/4) sqrt(pi)
    mu = moments(Fraction(2, 3), 4, mant_bits=128)
    assert mu[1].to_fraction() == 3
    with mpmath.workprec(200):
        v = mpmath.ldexp(mpmath.mpf(mu[0].M), mu[0].e)
        assert abs(v - mpmath.mpf(3) / 4 * mpmath.sqrt(mpmath.pi)) < mpmath.mpf(2) ** -125


def test_derivative_matches_finite_difference():
    beta = Fraction(1, 2)
    d = dmoments_dbeta(beta, 12, mant_bits=200)
    with mpmath.workprec(300):
        for j in range(12):
            f = lambda b: mpmath.gamma((j + 1) / b) / b
            ref = mpmath.diff(f, mpmath.mpf(1) / 2)
            val = mpmath.ldexp(mpmath.mpf(d[j].M), d[j].e)
            assert abs(val / ref - 1) < mpmath.mpf(2) ** -150


def test_limb_round_trip():
    vals = [0, 1, 2**32 - 1, 2**32, 3**200, 2**511 + 12345]
    arr = pack_limbs(vals, 16)
    assert unpack_limbs(arr) == vals
    neg = [(-5) % (1 << 512), (-(3**100)) % (1 << 512)]
    assert unpack_limbs(pack_limbs(neg, 16), signed=True) == [-5, -(3**100)]


def test_batch_configs_seeded_and_in_range():
    a = batch_configs()
    b = batch_configs()
    assert a == b and len(a) == 64
    for beta, N, P in a:
        assert beta in (Fraction(1, 3), Fraction(1, 2), Fraction(2, 3), Fraction(1))
        assert 32 <= N <= 512 and P % 128 == 0 and P >= 512


def test_precision_rule_beta_half_matches_condition_estimate():
    # Section 2.1: cond(H_N) ~ 20 Gamma(4N - 2) at beta = 1/2
    N = 100
    est = math.lgamma(4 * N - 2) / math.log(2) + math.log2(20)
    P = precision_rule(Fraction(1, 2), N)
    assert est + 512 <= P + 2 and P < est + 512 + 130


def test_float_beta_is_its_exact_decimal_or_refused():
    from hankel_inputs.moments import _as_fraction
    assert _as_fraction(0.45) == Fraction(9, 20)
    assert _as_fraction(0.5) == Fraction(1, 2)
    assert _as_fraction(0.123456) == Fraction(123456, 10**6)
    # a decimal that would need a larger denominator is refused, not snapped
    with pytest.raises(ValueError):
        _as_fraction(0.1234567891)
