"""Device-detected errors come back as status words, with the index the
contract names, and leave the library usable.

* EOVERFLOW at a factor column: a non-positive-definite Hankel input whose
  column 0 factor u_1 = rnd(a_10 / 2^h_0) exceeds 3 * 2^(P-3) (Algorithm 1's
  B_i = A_i / A_i[i] with A_i[i] tiny), the same code and column as the oracle.
* EOVERFLOW at the load: a moment above the scale bound of its row
  (bitlen(a_rc) > W + 1), reported at that row.
* Precision below the need of the matrix (beta = 1/2, N = 192 at P = 256 bits):
  the GPU reports the oracle's code and index.
* ENOCONV: the eigen-step given one iteration per block (hl_set_eig_maxit),
  reported for block 0 by hl_lambda_min and hl_lambda_min_noalloc; the default
  limit afterwards gives lambda_1 again.
No kernel faults: every error is a status word the kernels set and return on."""
from fractions import Fraction

import pytest

from hankel_inputs import Dyadic, moments
from oracle import contract as C

from gpu_util import ctx, say

pytestmark = pytest.mark.gpu


def overflow_moments():
    # E = 2: rows 0, 1 share s = ceil(41 / 2) = 21 from mu_2 = 2^40; mu_1 = 2^23
    # exceeds sqrt(mu_0 mu_2) = 2^20, so u_1 = 2^P at P bits
    return [Dyadic(1, 0), Dyadic(1, 23), Dyadic(1, 40), Dyadic(1, 30), Dyadic(1, 60)]


def oracle_error(mu, N, P, E):
    with pytest.raises(C.ContractError) as e:
        C.factor(mu, N, P, E)
    return e.value.code, e.value.index


@pytest.mark.parametrize("form", ["valu", "mfma"])
def test_eoverflow_at_factor_column(form):
    from paper_1810_01478_amd._lib import HLError, HL_EOVERFLOW
    mu = overflow_moments()
    assert oracle_error(mu, 3, 256, 2) == (C.EOVERFLOW, 0)
    say("EOVERFLOW column, form", form)
    fac = ctx().factor(mu, 3, 1, 256, 2, form)
    with pytest.raises(HLError) as e:
        ctx().sync(fac)
    assert e.value.code == HL_EOVERFLOW and "(index 0)" in str(e.value)


def test_eoverflow_at_load_row():
    from paper_1810_01478_amd._lib import HLError, HL_EOVERFLOW
    # E = 1: s_r = ceil(bitlen(mu_2r) / 2) = 1 for r = 0, 1, 2; a_10 = 2^40 2^(W - 2)
    # has bitlen W + 39 > W + 1
    mu = [Dyadic(1, 0), Dyadic(1, 40), Dyadic(1, 0), Dyadic(1, 0), Dyadic(1, 0)]
    say("EOVERFLOW load")
    fac = ctx().factor(mu, 3, 1, 256, 1, "valu")
    with pytest.raises(HLError) as e:
        ctx().sync(fac)
    assert e.value.code == HL_EOVERFLOW and "(index 1)" in str(e.value)


@pytest.mark.parametrize("form", ["valu", "mfma"])
def test_precision_too_low_matches_oracle(form):
    from paper_1810_01478_amd._lib import HLError
    N, P, E = 192, 256, 16
    mu = moments(Fraction(1, 2), 2 * N - 1)
    code, idx = oracle_error(mu, N, P, E)
    say("precision too low, oracle code", code, "index", idx, "form", form)
    fac = ctx().factor(mu, N, 1, P, E, form)
    with pytest.raises(HLError) as e:
        ctx().sync(fac)
    assert e.value.code == code and "(index %d)" % idx in str(e.value)


def test_enoconv_from_iteration_limit_then_recovers():
    from paper_1810_01478_amd._lib import HLError, HL_ENOCONV
    c = ctx()
    N, k, P, E = 64, 8, 2048, 16
    mu = moments(Fraction(1, 2), 2 * N - 1)
    fac = c.factor(mu, N, k, P, E, "mfma")
    c.inv_block(fac)
    try:
        c.set_eig_maxit(1)
        say("ENOCONV, hl_lambda_min")
        with pytest.raises(HLError) as e:
            c.eigen(fac)
        assert e.value.code == HL_ENOCONV and "index 0" in str(e.value)
        say("ENOCONV, hl_lambda_min_noalloc")
        with pytest.raises(HLError) as e:
            c.eigen_noalloc(fac)
        assert e.value.code == HL_ENOCONV and "index 0" in str(e.value)
    finally:
        c.set_eig_maxit(0)
    # the workspace's status word still holds ENOCONV: a fresh factorisation
    # and the default limit give lambda_1
    fac = c.factor(mu, N, k, P, E, "mfma")
    res = c.lambda_min(fac)
    assert res["lambda1"] > 0 and res["iterations"] > 2
    assert c.eigen_noalloc(fac)["lambda1"] == res["lambda1"]
