"""The leading-exponent fit of Section 6 ("Linear fit").

CPU: the oracle (oracle/fit.py) is pinned by the numbers Section 6 prints for
Table 2's lambda_1 (slope 0.63646, intercept 0.04630, adjusted R-squared
0.999997, the interval [0.63510, 0.63781], which is the 99% Student-t interval),
by exact recovery of a line, and by closed-form t quantiles (1 and 2 degrees of
freedom) and textbook ones; planted mistakes (weights N instead of N^2, a
dropped sqrt(log N)) fail the pin.  The product fit
(paper_1810_01478_amd.exponent_fit, numpy + scipy) equals the oracle on Table 2
and on seeded synthetic data.
GPU: lambda_1 recomputed at N = 500 .. 2000 gives the fit of Table 2's values."""
import math
from fractions import Fraction

import mpmath
import numpy as np
import pytest

from golden_table2 import table2
from oracle import fit as F


def _table():
    t = table2()
    N = sorted(t)
    return N, [t[n].lambda1 for n in N]


def test_oracle_reproduces_section6():
    N, lam = _table()
    o = F.line(N, lam)
    assert round(float(o.slope), 5) == 0.63646
    assert round(float(o.intercept), 5) == 0.04630
    assert round(float(o.adj_r2), 6) == 0.999997
    lo, hi = F.interval(o, 0.99)
    assert (round(float(lo), 5), round(float(hi), 5)) == (0.63510, 0.63781)
    lo95, hi95 = F.interval(o, 0.95)
    assert lo95 < 2 / math.pi < hi95 and lo < 2 / math.pi < hi
    # the relative distance to 2/pi as Section 6 forms it from the rounded values
    assert round((0.63662 - round(float(o.slope), 5)) / 0.63662, 5) == 0.00025


def test_oracle_exact_line():
    # points placed exactly on y = a + b x are fitted exactly
    a, b = mpmath.mpf("0.125"), mpmath.mpf("0.6")
    N = [300, 700, 1100, 2500, 4000]
    with mpmath.workprec(300):
        lam = [8 * mpmath.pi * mpmath.sqrt(mpmath.log(n)) / mpmath.exp(a + b * mpmath.log(4 * mpmath.pi * n * mpmath.e))
               for n in N]
        o = F.line(N, lam, prec=300)
        assert abs(o.slope - b) < mpmath.mpf(10) ** -60
        assert abs(o.intercept - a) < mpmath.mpf(10) ** -60
        assert max(abs(r) for r in o.residuals) < mpmath.mpf(10) ** -60


def test_t_quantiles():
    with mpmath.workprec(200):
        for p in ("0.9", "0.975", "0.995"):
            pm = mpmath.mpf(p)
            # one degree of freedom: Cauchy, t = tan(pi (p - 1/2))
            assert abs(F.t_quantile(pm, 1) - mpmath.tan(mpmath.pi * (pm - mpmath.mpf(1) / 2))) < mpmath.mpf(10) ** -30
            # two: t = (2p - 1) / sqrt(2 p (1 - p))
            assert abs(F.t_quantile(pm, 2) - (2 * pm - 1) / mpmath.sqrt(2 * pm * (1 - pm))) < mpmath.mpf(10) ** -30
    # textbook table values (three decimals)
    for p, nu, v in ((0.975, 7, 2.365), (0.995, 7, 3.499), (0.975, 30, 2.042), (0.95, 10, 1.812)):
        assert abs(float(F.t_quantile(p, nu)) - v) < 5e-4


@pytest.mark.parametrize("mutation", ["weights_N", "no_sqrt_log"])
def test_planted_fit_mistakes_are_caught(mutation):
    N, lam = _table()
    if mutation == "weights_N":
        o = F.line(N, lam, weight_power=1)
    else:
        # y without the sqrt(log N) factor: fit log(8 pi / lambda_1) instead
        lam2 = [l / math.sqrt(math.log(n)) for n, l in zip(N, lam)]
        o = F.line(N, lam2)
    assert round(float(o.slope), 5) != 0.63646


def test_product_fit_matches_oracle():
    from paper_1810_01478_amd.exponent_fit import fit
    rng = np.random.default_rng(1810)
    cases = [_table()]
    for _ in range(3):
        N = sorted(int(v) for v in rng.choice(np.arange(200, 5000), size=12, replace=False))
        lam = [8 * math.pi * math.sqrt(math.log(n)) / (4 * math.pi * n * math.e) ** (2 / math.pi)
               * (1 + 0.3 / math.log(n) + 1e-3 * rng.standard_normal()) for n in N]
        cases.append((N, lam))
    for N, lam in cases:
        for wp in (0, 2):
            g = fit(N, lam, weight_power=wp)
            o = F.line(N, lam, weight_power=wp)
            assert abs(g["slope"] / float(o.slope) - 1) < 1e-10
            assert abs(g["intercept"] - float(o.intercept)) < 1e-10
            assert abs(g["se_slope"] / float(o.se_slope) - 1) < 1e-8
            assert abs(g["adj_r2"] - float(o.adj_r2)) < 1e-10
            for level in (95, 99):
                lo, hi = F.interval(o, level / 100)
                assert abs(g["ci%d" % level][0] - float(lo)) < 1e-10
                assert abs(g["ci%d" % level][1] - float(hi)) < 1e-10


@pytest.mark.gpu
def test_fit_on_gpu_lambdas():
    from paper_1810_01478_amd import table2 as T
    from paper_1810_01478_amd.exponent_fit import fit
    from gpu_util import ctx, say
    t = table2()
    Ns = [500, 1000, 1500, 2000]
    lam = []
    for N in Ns:
        # two steps above the paper's required precision
        r = T.run_at(ctx(), Fraction(1, 2), N, 8, t[N].K_bits + 2048, E=1, form="mfma", count=0)
        assert "error" not in r, r
        say("fit point", N, r["P"], r["lambda"][0])
        lam.append(r["lambda"][0])
    g = fit(Ns, lam)
    ref = F.line(Ns, [t[n].lambda1 for n in Ns])
    say("  slope", g["slope"], "from Table 2", float(ref.slope))
    # lambda_1 agrees with the printed values to ~1e-15, so the fit does to ~1e-13
    assert abs(g["slope"] / float(ref.slope) - 1) < 1e-11
    assert abs(g["intercept"] - float(ref.intercept)) < 1e-11
