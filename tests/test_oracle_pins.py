"""Pins of the CPU oracle against facts that do not come from the oracle itself.

* closed forms at beta = 1 (mu_j = j!): D_m = (m!)^2 and L_ri = C(r,i) r!/i!
  exactly, det H_N = prod (m!)^2;
* exact rational LDL^T for tiny N (beta = 1/2, irrational-free but with
  non-integer factors), within the contract's rounding bound;
* the brute-force characteristic polynomial for N <= 8 (sympy's independent
  routine and the Sturm-isolated smallest root, and the second and third
  roots for lambda_2 and lambda_3);
* the values printed in Table 2 at N = 500;
* agreement at doubled precision;
* interlacing (trunc <= 0), positivity of pivots, the error paths.
"""
import math
from fractions import Fraction

import mpmath
import pytest

from hankel_inputs import moments
from oracle import contract as C
from oracle import exact as X


def _mu(beta, N, bits=0):
    return moments(beta, 2 * N - 1, mant_bits=bits)


# ------------------------------------------------------------------ beta = 1 closed forms

@pytest.mark.parametrize("N,P", [(32, 2048), (64, 4096)])
def test_beta1_pivots_and_multipliers_closed_form(N, P):
    f = C.factor(_mu(1, N), N, P, E=16)
    W = f.W
    for m in range(N):
        assert f.d[m] == math.factorial(m) ** 2 << (W - 2 * f.s[m])
    for i in range(N):
        for r in range(i + 1, N):
            L = math.comb(r, i) * math.factorial(r) // math.factorial(i)
            ex = f.s[i] + f.h[i] - f.s[r]
            assert ex >= 0
            assert f.b[i][r] == L << ex


def test_exact_ldl_beta1_and_determinant():
    N = 9
    H = X.hankel([m.to_fraction() for m in _mu(1, N)], N)
    L, D = X.ldl(H)
    assert D == [Fraction(math.factorial(m) ** 2) for m in range(N)]
    for r in range(N):
        for i in range(r):
            assert L[r][i] == math.comb(r, i) * Fraction(math.factorial(r), math.factorial(i))
    # det H_N = prod D = prod (m!)^2, against sympy's determinant
    import sympy
    det = sympy.Matrix([[sympy.Integer(int(v)) for v in row] for row in H]).det()
    assert det == math.prod(math.factorial(m) ** 2 for m in range(N))


def test_exact_linv_beta1_closed_form():
    # (L^-1)_ij = (-1)^(i-j) C(i,j) i!/j! for the Laguerre moments
    N = 9
    H = X.hankel([m.to_fraction() for m in _mu(1, N)], N)
    L, D = X.ldl(H)
    Xi = X.linv_cols(L, 4)
    for a in range(4):
        for r in range(N):
            want = 0 if r < a else (-1) ** (r - a) * math.comb(r, a) * Fraction(math.factorial(r), math.factorial(a))
            assert Xi[r][a] == want


# ------------------------------------------------------------------ exact rationals, beta = 1/2

@pytest.mark.parametrize("N,P,E", [(12, 1024, 1), (20, 2048, 16), (24, 2048, 4)])
def test_contract_matches_exact_rationals(N, P, E):
    mu = _mu(Fraction(1, 2), N)
    f = C.factor(mu, N, P, E)
    H = X.hankel([m.to_fraction() for m in mu], N)
    L, D = X.ldl(H)
    for i in range(N):
        rel = abs(C.D_value(f, i) / D[i] - 1)
        assert rel < Fraction(1, 2 ** (P // 2)), (i, float(rel))
    for i in range(N):
        for r in range(i + 1, N):
            assert abs(C.L_value(f, r, i) - L[r][i]) <= abs(L[r][i]) * Fraction(1, 2 ** (P // 2)) + Fraction(1, 2 ** (P // 2))


def test_block_matches_exact_hinv():
    N, P, k = 16, 2048, 6
    mu = _mu(Fraction(1, 2), N)
    f = C.factor(mu, N, P, 16)
    sv = C.solve(f, k)
    bl = C.block(f, sv)
    H = X.hankel([m.to_fraction() for m in mu], N)
    L, D = X.ldl(H)
    Hi = X.hinv_block(X.linv_cols(L, k), D, k)
    scale = Fraction(2) ** bl.blk_exp if bl.blk_exp >= 0 else Fraction(1, 2 ** -bl.blk_exp)
    top = max(abs(v) for row in Hi for v in row)
    for a in range(k):
        for b in range(k):
            assert abs(bl.blk[a][b] * scale - Hi[a][b]) <= top * Fraction(1, 2 ** (P // 2))


# ------------------------------------------------------------------ brute-force characteristic polynomial

@pytest.mark.parametrize("beta", [Fraction(1, 2), Fraction(1), Fraction(1, 3)])
@pytest.mark.parametrize("N", [4, 8])
def test_lambda1_against_characteristic_polynomial(beta, N):
    mu = _mu(beta, N)
    H = X.hankel([m.to_fraction() for m in mu], N)
    c = X.charpoly(H)
    import sympy
    x = sympy.symbols("x")
    sp = sympy.Matrix([[sympy.Rational(v.numerator, v.denominator) for v in row] for row in H]).charpoly(x).all_coeffs()[::-1]
    assert [Fraction(int(sympy.numer(v)), int(sympy.denom(v))) for v in sp] == c
    tr = sum(H[i][i] for i in range(N))
    lam = X.smallest_root(c, tr, bits=400 + int(tr).bit_length())
    P = 1024
    f, sv, bl, ev = C.lambda_min(mu, N, N, P, E=1)   # k = N: the block is all of H^-1
    with mpmath.workprec(600):
        ref = mpmath.mpf(lam.numerator) / lam.denominator
        assert abs(ev.lam1 / ref - 1) < mpmath.mpf(10) ** -90


def _polymul(a, b):
    out = [Fraction(0)] * (len(a) + len(b) - 1)
    for i, x in enumerate(a):
        for j, y in enumerate(b):
            out[i + j] += x * y
    return out


def test_kth_root_known_roots():
    roots = [Fraction(1, 3), Fraction(2), Fraction(7, 2), Fraction(10)]
    c = [Fraction(1)]
    for r in roots:
        c = _polymul(c, [-r, Fraction(1)])   # coefficients low to high
    for j, r in enumerate(roots, start=1):
        got = X.kth_root(c, j, Fraction(16), bits=200)
        assert abs(got - r) <= Fraction(16, 2 ** 199)
    assert X.kth_root(c, 1, Fraction(16), bits=200) == X.smallest_root(c, Fraction(16), bits=200)
    with pytest.raises(ValueError):
        X.kth_root(c, 4, Fraction(5))


@pytest.mark.parametrize("beta", [Fraction(1, 2), Fraction(1), Fraction(1, 3)])
@pytest.mark.parametrize("N", [4, 8])
def test_next_eigenvalues_against_characteristic_polynomial(beta, N):
    # k = N: the block is all of H^-1, so lambda_2 and lambda_3 are the second
    # and third roots of the characteristic polynomial, isolated exactly
    mu = _mu(beta, N)
    H = X.hankel([m.to_fraction() for m in mu], N)
    c = X.charpoly(H)
    tr = sum(H[i][i] for i in range(N))
    P = 1024
    f, sv, bl, ev = C.lambda_min(mu, N, N, P, E=1)
    nxt = C.eigen_next(bl, 2, P=P)
    assert [r.j for r in nxt] == [2, 3]
    with mpmath.workprec(600):
        for r in nxt:
            root = X.kth_root(c, r.j, tr, bits=400 + int(tr).bit_length())
            ref = mpmath.mpf(root.numerator) / root.denominator
            assert abs(r.lam / ref - 1) < mpmath.mpf(10) ** -90
            assert r.trunc <= 0
        assert ev.lam1 < nxt[0].lam < nxt[1].lam


@pytest.mark.parametrize("mutation", ["ascending", "off_by_one"])
def test_planted_eigen_next_mistakes_are_caught(monkeypatch, mutation):
    # the real _eigs_desc passes the characteristic-polynomial pin; an ordering
    # or index mistake in it must not
    N, P = 6, 1024
    mu = _mu(Fraction(1, 2), N)
    H = X.hankel([m.to_fraction() for m in mu], N)
    c = X.charpoly(H)
    tr = sum(H[i][i] for i in range(N))
    root = X.kth_root(c, 2, tr, bits=400 + int(tr).bit_length())
    _, _, bl, _ = C.lambda_min(mu, N, N, P, E=1)
    real = C._eigs_desc
    if mutation == "ascending":
        monkeypatch.setattr(C, "_eigs_desc", lambda m, p: real(m, p)[::-1])
    else:
        monkeypatch.setattr(C, "_eigs_desc", lambda m, p: real(m, p)[1:] + real(m, p)[:1])
    lam2 = C.eigen_next(bl, 1, P=P)[0].lam
    with mpmath.workprec(600):
        ref = mpmath.mpf(root.numerator) / root.denominator
        assert abs(lam2 / ref - 1) > mpmath.mpf(10) ** -10


def test_next_eigenvalues_bad_count():
    mu = _mu(Fraction(1, 2), 16)
    _, _, bl, _ = C.lambda_min(mu, 16, 3, 1024, 16)
    C.eigen_next(bl, 1, P=1024)
    with pytest.raises(C.ContractError):
        C.eigen_next(bl, 2, P=1024)       # the 2 x 2 leading block has no third eigenvalue
    with pytest.raises(C.ContractError):
        C.eigen_next(bl, 0, P=1024)


# ------------------------------------------------------------------ doubled precision, full-matrix eigenvalues

def test_doubled_precision_agreement_c1():
    mu = _mu(Fraction(1, 2), 64)
    _, _, _, a = C.lambda_min(mu, 64, 8, 2048, 16)
    _, _, _, b = C.lambda_min(mu, 64, 8, 4096, 16)
    with mpmath.workprec(9000):
        assert abs(a.lam1 / b.lam1 - 1) < mpmath.mpf(10) ** -300
        assert a.trunc <= 0 and b.trunc <= 0
        assert abs(a.trunc / b.trunc - 1) < mpmath.mpf(10) ** -200


def test_truncation_against_full_matrix_eigenvalue():
    # untruncated lambda_1 of H_32 by a dense eigen-solver on the exact matrix
    N = 32
    mu = _mu(Fraction(1, 2), N)
    with mpmath.workprec(1500):
        M = mpmath.matrix(N, N)
        for i in range(N):
            for j in range(N):
                M[i, j] = mpmath.mpf(mu[i + j].M)
        lam_full = min(mpmath.eigsy(M, eigvals_only=True))
    _, _, _, ev_full = C.lambda_min(mu, N, N, 2048, 16)
    _, _, _, ev8 = C.lambda_min(mu, N, 8, 2048, 16)
    with mpmath.workprec(1500):
        assert abs(ev_full.lam1 / lam_full - 1) < mpmath.mpf(10) ** -100
        err8 = ev8.lam1 - lam_full
        assert err8 >= 0                      # truncating H^-1 can only raise 1/lambda_max
        assert err8 < abs(ev8.trunc) * 10     # the k-1 difference bounds the k error


def test_next_truncation_against_full_matrix_eigenvalues():
    # lambda_2, lambda_3 of H_32 by a dense eigen-solver on the exact matrix:
    # k = N reproduces them; k = 8 can only raise them (Poincare separation:
    # the j-th eigenvalue of a compression of H^-1 is at most that of H^-1)
    N = 32
    mu = _mu(Fraction(1, 2), N)
    with mpmath.workprec(1500):
        M = mpmath.matrix(N, N)
        for i in range(N):
            for j in range(N):
                M[i, j] = mpmath.mpf(mu[i + j].M)
        full = sorted(mpmath.eigsy(M, eigvals_only=True)[i] for i in range(N))
    _, _, bl_full, _ = C.lambda_min(mu, N, N, 2048, 16)
    _, _, bl8, _ = C.lambda_min(mu, N, 8, 2048, 16)
    nf = C.eigen_next(bl_full, 2, P=2048)
    n8 = C.eigen_next(bl8, 2, P=2048)
    with mpmath.workprec(1500):
        for r_full, r8 in zip(nf, n8):
            ref = full[r_full.j - 1]
            assert abs(r_full.lam / ref - 1) < mpmath.mpf(10) ** -100
            err = r8.lam - ref
            assert err >= 0
            assert r8.trunc <= 0
            assert err < abs(r8.trunc) * 10


# ------------------------------------------------------------------ Table 2

@pytest.mark.slow
def test_table2_n500():
    # Table 2, N = 500, beta = 1/2: smallest eigenvalue 0.1204653471966412 with
    # truncation error -6.52e-16 (k = 8; the paper reports 16 digits from a
    # double-precision eigen-solve, so 1e-15 relative is the comparison bar).
    mu = _mu(Fraction(1, 2), 500)
    _, _, bl, ev = C.lambda_min(mu, 500, 8, 1280, E=1)
    assert abs(float(ev.lam1) / 0.1204653471966412 - 1) < 1e-15
    assert -7.5e-16 < float(ev.trunc) < -5.5e-16
    # lambda_2 and lambda_3 (Table 2's other columns) within the error of the
    # paper's double-precision eigen-solve (tests/golden_table2.paper_error)
    from golden_table2 import paper_error, table2
    row = table2()[500]
    for r in C.eigen_next(bl, 2, P=1280):
        e_lam, e_tr = paper_error(row, r.j)
        assert abs(float(r.lam) - (row.lambda2, row.lambda3)[r.j - 2]) <= e_lam
        assert float(r.trunc) < 0
        assert abs(float(r.trunc) - (row.trunc2, row.trunc3)[r.j - 2]) <= e_tr


# ------------------------------------------------------------------ invariants and error paths

def test_pivots_positive_and_reconstruction():
    N, P = 24, 1024
    mu = _mu(Fraction(1, 2), N)
    f = C.factor(mu, N, P, 4)
    assert all(v > 0 for v in f.d)
    H = X.hankel([m.to_fraction() for m in mu], N)
    for r in range(N):
        for c in range(r + 1):
            v = sum((C.L_value(f, r, i) if r != i else 1) * C.D_value(f, i) * (C.L_value(f, c, i) if c != i else 1)
                    for i in range(c + 1))
            assert abs(v / H[r][c] - 1) < Fraction(1, 2 ** (P // 2))


def test_not_positive_definite_input():
    # mu_2 < mu_1^2 / mu_0 breaks positive definiteness at pivot 1
    from hankel_inputs import Dyadic
    mu = [Dyadic(4, 0), Dyadic(4, 0), Dyadic(3, 0), Dyadic(9, 0), Dyadic(30, 0)]
    with pytest.raises(C.ContractError) as e:
        C.factor(mu, 3, 256, 1)
    assert e.value.code == C.ENOTPD and e.value.index == 1


def test_precision_too_small_is_reported():
    mu = _mu(Fraction(1, 2), 64)
    with pytest.raises(C.ContractError) as e:
        C.factor(mu, 64, 128, 16)
    assert e.value.code in (C.ENOTPD, C.EOVERFLOW)


def test_bad_arguments():
    with pytest.raises(C.ContractError) as e:
        C.factor(_mu(1, 4), 4, 100, 1)
    assert e.value.code == C.EINVAL


def test_right_and_left_looking_agree_bit_for_bit():
    # the update is exact, so a left-looking order (all earlier columns applied
    # to column i just before it is factored) must give identical d, h, b
    N, P, E = 40, 1024, 8
    mu = _mu(Fraction(1, 2), N)
    f = C.factor(mu, N, P, E)
    s = C.scales(mu, N, E)
    A = C.load(mu, N, P, s)
    d, h, B, U = [], [], [], []
    for i in range(N):
        col = [A[r][i] if r >= i else None for r in range(N)]
        for j in range(i):
            for r in range(i, N):
                col[r] -= B[j][r] * U[j][i]
        di = col[i]
        hi, wi = C.pivot_reciprocal(di, P)
        u = {r: C.rnd_shift(col[r], hi) for r in range(i + 1, N)}
        b = {r: C.rnd_shift(u[r] * wi, P) for r in range(i + 1, N)}
        u[i] = 0
        d.append(di); h.append(hi); B.append(b); U.append(u)
    assert d == f.d and h == f.h and B == f.b


# ------------------------------------------------------------------ rounding helpers and planted mistakes

def test_rounding_helpers_against_fractions():
    import random
    rng = random.Random(7)
    for _ in range(2000):
        a = rng.randrange(-(1 << 200), 1 << 200)
        d = rng.randrange(1, 1 << 120)
        q = C.rnd_div(a, d)
        fr = Fraction(a, d)
        assert abs(fr - q) <= Fraction(1, 2)
        if abs(fr - q) == Fraction(1, 2):
            assert abs(q) > abs(fr)            # ties away from zero
        s = rng.randrange(1, 90)
        q2 = C.rnd_shift(a, s)
        fr2 = Fraction(a, 1 << s)
        assert abs(fr2 - q2) <= Fraction(1, 2)
        if abs(fr2 - q2) == Fraction(1, 2):
            assert abs(q2) > abs(fr2)
    assert C.rnd_shift(5, 1) == 3 and C.rnd_shift(-5, 1) == -3 and C.rnd_shift(3, -2) == 12


@pytest.mark.parametrize("mutation", ["sign", "index", "no_scale"])
def test_planted_mistakes_are_caught(monkeypatch, mutation):
    """A copy of the factor loop with one plausible mistake must fail the
    closed-form / exact-rational pins that the real oracle passes."""
    N, P = 12, 1024
    mu = _mu(1, N)
    s = C.scales(mu, N, 4)
    # "no_scale": one global binary point instead of the per-row scales
    A = C.load(mu, N, P, s if mutation != "no_scale" else [max(s)] * N)
    d = []
    for i in range(N):
        di = A[i][i]
        if di <= 0:          # the mistake already broke positive definiteness
            d.append(di)
            break
        hi, wi = C.pivot_reciprocal(di, P)
        u = {r: C.rnd_shift(A[r][i], hi) for r in range(i + 1, N)}
        b = {r: C.rnd_shift(u[r] * wi, P) for r in range(i + 1, N)}
        for c in range(i + 1, N):
            for r in range(c, N):
                if mutation == "sign":
                    A[r][c] += b[r] * u[c]
                elif mutation == "index":
                    A[r][c] -= b[c] * u[c]
                else:
                    A[r][c] -= b[r] * u[c]
        d.append(di)
    W = 2 * P - 4
    ok = all(d[m] == math.factorial(m) ** 2 << (W - 2 * C.scales(mu, N, 4)[m]) for m in range(N))
    assert not ok


def _round_fraction(x: Fraction) -> int:
    # nearest integer, ties away from zero, from the definition (floor of x + 1/2
    # for x >= 0), independent of the oracle's rounding helpers
    assert x >= 0
    return math.floor(x + Fraction(1, 2))


@pytest.mark.parametrize("P", [256, 2048])
def test_pivot_reciprocal_is_the_rounded_quotient(P):
    # w = rnd(2^(2h+P) / d) with the whole pivot, h = floor(bitlen(d) / 2), on
    # random pivots and on pivots whose quotient sits within 2^-60 of a tie
    from recip_cases import near_tie_pivots, random_pivots
    for d in random_pivots(P, 200, P) + near_tie_pivots(P, 200, P + 1):
        h, w = C.pivot_reciprocal(d, P)
        L = 0
        while (1 << L) <= d:
            L += 1
        assert h == L // 2
        assert w == _round_fraction(Fraction(1 << (2 * h + P), d))
        assert (1 << (P - 1)) <= w <= (1 << (P + 1))


def test_planted_cut_reciprocal_fails_near_ties():
    # a reciprocal taken from d cut to its top P + 64 bits agrees on random
    # pivots but not on every near-tie pivot: the near-tie cases pin the
    # definition where the two readings differ
    from recip_cases import near_tie_pivots
    P = 256
    differ = 0
    for d in near_tie_pivots(P, 400, 5):
        h, w = C.pivot_reciprocal(d, P)
        m = max(0, d.bit_length() - P - 64)
        cut = _round_fraction(Fraction(1 << (2 * h + P - m), d >> m))
        differ += cut != w
    assert differ > 0


def test_scales_by_hand_beta1():
    # beta = 1: mu_2j = (2j)!, whose bit lengths for j = 0..19 are
    # 1 2 5 10 | 16 22 29 37 | 45 53 62 70 | 80 89 98 108 | 118 128 139 149;
    # with E = 4 the block maxima are 10, 37, 70, 108, 149 and s = ceil(t / 2)
    N, E = 20, 4
    mu = _mu(1, N)
    bl = [1, 2, 5, 10, 16, 22, 29, 37, 45, 53, 62, 70, 80, 89, 98, 108, 118, 128, 139, 149]
    assert [math.factorial(2 * j).bit_length() for j in range(N)] == bl
    assert C.scales(mu, N, E) == [5] * 4 + [19] * 4 + [35] * 4 + [54] * 4 + [75] * 4
    # E = 1: every row its own ceil(bitlen / 2); E = 7: ragged last block
    assert C.scales(mu, N, 1) == [1, 1, 3, 5, 8, 11, 15, 19, 23, 27, 31, 35, 40, 45, 49, 54, 59, 64, 70, 75]
    assert C.scales(mu, N, 7) == [15] * 7 + [45] * 7 + [75] * 6
    # dyadic exponents count: mu * 2^-9 lowers every bit length by 9
    from hankel_inputs import Dyadic
    mu9 = [Dyadic(m.M, m.e - 9) for m in mu]
    assert C.scales(mu9, N, E) == [1] * 4 + [14] * 4 + [31] * 4 + [50] * 4 + [70] * 4


@pytest.mark.parametrize("mutation", ["floor", "block_shift"])
def test_planted_scale_mistakes_are_caught(monkeypatch, mutation):
    orig = C.scales

    def bad(mu, N, E):
        if mutation == "floor":
            t = [C.bitlen(mu[2 * j].M, mu[2 * j].e) for j in range(N)]
            out = []
            for j0 in range(0, N, E):
                tJ = max(t[j0:j0 + E])
                out.extend([tJ // 2] * (min(N, j0 + E) - j0))
            return out
        s = orig(mu, N, E)
        return s[1:] + s[-1:]
    monkeypatch.setattr(C, "scales", bad)
    N, E = 20, 4
    assert C.scales(_mu(1, N), N, E) != [5] * 4 + [19] * 4 + [35] * 4 + [54] * 4 + [75] * 4
