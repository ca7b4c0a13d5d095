"""Pins of the oracle's GMP back-end and of its row-parallel runner.

* oracle.gmp against Python's own integers (an independent implementation of
  the same exact arithmetic);
* oracle.parallel against the single-process contract, bit for bit: pivots,
  exponents, reciprocals, the digest of every multiplier column, X, the block
  and lambda_1, on several shapes and process counts, and on the error paths.
"""
import random
from fractions import Fraction

import pytest

from hankel_inputs import Dyadic, moments
from oracle import contract as C
from oracle import gmp as G
from oracle import parallel as PAR

pytestmark = pytest.mark.skipif(not G.available(), reason="libgmp not loadable")


def test_gmp_submul_addmul_against_python_ints():
    rng = random.Random(3)
    for bits in (1, 31, 64, 65, 1000, 8192, 49152, 200000):
        for _ in range(4):
            a = rng.getrandbits(2 * bits) * rng.choice((-1, 1))
            b = rng.getrandbits(bits) * rng.choice((-1, 1))
            u = rng.getrandbits(bits) * rng.choice((-1, 1, 0))
            assert G.submul_int(a, b, u) == a - b * u
            x = G.Mpz(a)
            x.addmul(G.Mpz(b), G.Mpz(u))
            assert x.get() == a + b * u
    assert G.Mpz(0).get() == 0
    z = G.Mpz(5)
    raw = (12345678901234567890).to_bytes(16, "little")
    import ctypes
    buf = ctypes.create_string_buffer(raw, 16)
    z.set_bytes(ctypes.addressof(buf), 16, True)
    assert z.get() == -12345678901234567890


def test_contract_with_gmp_submul_hook():
    N, P, E = 24, 512, 4
    mu = moments(Fraction(1, 2), 2 * N - 1)
    f0 = C.factor(mu, N, P, E)
    f1 = C.factor(mu, N, P, E, submul=G.submul_int)
    assert f0.d == f1.d and f0.b == f1.b and f0.h == f1.h and f0.w == f1.w


@pytest.mark.parametrize("beta,N,P,E,k,nproc", [
    (Fraction(1, 2), 40, 1024, 16, 8, 3),
    (Fraction(1, 2), 33, 1024, 5, 6, 1),
    (Fraction(1, 3), 30, 1536, 1, 30, 4),
    (1, 20, 512, 4, 1, 8),
])
def test_parallel_equals_contract(beta, N, P, E, k, nproc):
    mu = moments(beta, 2 * N - 1)
    f = C.factor(mu, N, P, E)
    sv = C.solve(f, k)
    bl = C.block(f, sv)
    ev = C.eigen(bl, P=P)
    pf = PAR.factor_solve(mu, N, P, E, k, nproc)
    assert pf.s == f.s and pf.d == f.d and pf.h == f.h and pf.w == f.w
    assert (pf.G, pf.Q) == (sv.G, sv.Q)
    assert pf.X == sv.X
    nl, nw = P // 32, P // 16
    assert pf.b_sha == [PAR.column_digest([f.b[i][r] for r in range(i + 1, N)], nl) for i in range(N - 1)]
    assert pf.d_sha == [PAR.column_digest([f.d[i]], nw) for i in range(N)]
    pbl = PAR.block(pf, nproc=2)
    assert pbl.blk == bl.blk and pbl.blk_exp == bl.blk_exp and pbl.Mt == bl.Mt
    pev = C.eigen(pbl, P=P)
    assert pev.lam1 == ev.lam1
    assert repr(pev.trunc) == repr(ev.trunc)   # nan for k = 1


def test_planted_update_mistake_changes_digests(monkeypatch):
    # a wrong sign in the exact update must show in the multiplier digests
    N, P, E, k = 16, 512, 4, 4
    mu = moments(Fraction(1, 2), 2 * N - 1)
    good = PAR.factor_solve(mu, N, P, E, k, 2)
    monkeypatch.setattr(G.Mpz, "submul", G.Mpz.addmul)
    try:
        bad = PAR.factor_solve(mu, N, P, E, k, 2)
    except C.ContractError:
        return  # the wrong update broke the factorisation outright
    assert bad.b_sha != good.b_sha


def test_parallel_not_positive_definite():
    mu = [Dyadic(4, 0), Dyadic(4, 0), Dyadic(3, 0), Dyadic(9, 0), Dyadic(30, 0)]
    with pytest.raises(C.ContractError) as e:
        PAR.factor_solve(mu, 3, 256, 1, 1, 2)
    assert e.value.code == C.ENOTPD and e.value.index == 1


def test_parallel_precision_too_small_matches_contract():
    mu = moments(Fraction(1, 2), 127)
    with pytest.raises(C.ContractError) as e0:
        C.factor(mu, 64, 128, 16)
    with pytest.raises(C.ContractError) as e1:
        PAR.factor_solve(mu, 64, 128, 16, 8, 3)
    assert (e1.value.code, e1.value.index) == (e0.value.code, e0.value.index)


def test_parallel_leading_columns_sample():
    N, P, E, k = 30, 1024, 8, 4
    mu = moments(Fraction(1, 2), 2 * N - 1)
    f = C.factor(mu, N, P, E)
    pf = PAR.factor_solve(mu, N, P, E, k, 3, columns=5)
    assert pf.d == f.d[:5] and pf.h == f.h[:5] and pf.w == f.w[:5]
    assert pf.b_sha == [PAR.column_digest([f.b[i][r] for r in range(i + 1, N)], P // 32) for i in range(5)]
