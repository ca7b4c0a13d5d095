"""GPU parity of hl_factor against the oracle: pivots d_i, balance exponents h_i,
scales s_j and multipliers b_ri must be bit-exact (the contract is exact integer
arithmetic with fixed rounding points)."""
import math
import random
from fractions import Fraction

import pytest

from hankel_inputs import moments
from oracle import contract as C

from gpu_util import ctx, say

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("na,nb", [(1, 1), (3, 5), (64, 64), (65, 63), (200, 131), (512, 514)])
def test_debug_mul_matches_host(na, nb):
    say("debug_mul", na, nb)
    rng = random.Random(na * 1000 + nb)
    for _ in range(4):
        a = rng.getrandbits(32 * na)
        b = rng.getrandbits(32 * nb)
        if rng.random() < 0.3:
            a = (1 << (32 * na)) - 1
            b = (1 << (32 * nb)) - 1
        got = ctx().debug_mul(a, b, na, nb, na + nb)
        assert got == a * b


def _structured(rng, n):
    """Random, all-ones, a power of two, runs of 0x7f bytes (the balanced-digit
    carry chains) and 0x80 bytes, for n limbs."""
    kind = rng.randrange(5)
    if kind == 0:
        return rng.getrandbits(32 * n)
    if kind == 1:
        return (1 << (32 * n)) - 1
    if kind == 2:
        return 1 << rng.randrange(32 * n)
    byte = 0x7f if kind == 3 else 0x80
    x = int.from_bytes(bytes([byte]) * (4 * n), "little")
    return x ^ (rng.getrandbits(8) << (8 * rng.randrange(4 * n)))


@pytest.mark.parametrize("na,nb,threads", [(1, 1, 256), (3, 5, 1024), (7, 7, 256), (8, 300, 1024), (64, 64, 256),
                                           (65, 63, 1024), (127, 135, 256), (200, 131, 256), (770, 1539, 1024),
                                           (1539, 1538, 1024)])
def test_debug_mul_wg_matches_host(na, nb, threads):
    # the one-workgroup MFMA product: exact, also truncated to fewer limbs
    say("debug_mul_wg", na, nb, threads)
    rng = random.Random(na * 7919 + nb)
    for it in range(5):
        a, b = _structured(rng, na), _structured(rng, nb)
        nout = na + nb if it % 2 == 0 else max(1, na + nb - rng.randrange(1, na + nb + 1))
        got = ctx().debug_mul_wg(a, b, na, nb, nout, threads)
        assert got == (a * b) % (1 << (32 * nout)), (it, nout)


@pytest.mark.parametrize("P", [256, 2048, 8192, 49152])
def test_debug_pivot_reciprocal(P):
    # w = rnd(2^(2h+P) / d) by the whole pivot: random pivots, and pivots whose
    # quotient lies within 2^-60 of a half-integer (where a reciprocal of d cut
    # to its top P + 64 bits can round the other way)
    from recip_cases import near_tie_pivots, random_pivots
    say("debug_recip", P)
    cases = random_pivots(P, 6, P) + near_tie_pivots(P, 10 if P < 49152 else 4, P + 1)
    for j, d in enumerate(cases):
        w, h = ctx().debug_recip(d, P)
        hh, ww = C.pivot_reciprocal(d, P)
        assert h == hh, j
        assert w == ww, (d.bit_length(), j)


def _check_factor(fac, f, N):
    assert fac.s_list() == f.s
    assert fac.h_list() == f.h
    piv = fac.pivots()
    assert piv == f.d
    for i in range(N - 1):
        assert fac.multipliers(i) == [f.b[i][r] for r in range(i + 1, N)], i


@pytest.mark.parametrize("beta,N,P,E,form", [
    (Fraction(1, 2), 64, 2048, 16, "valu"),
    (Fraction(1, 2), 80, 1024, 7, "valu"),
    (Fraction(1, 3), 45, 1536, 1, "valu"),
])
def test_factor_bit_exact_vs_oracle(beta, N, P, E, form):
    say("factor", beta, N, P, E, form)
    mu = moments(beta, 2 * N - 1)
    f = C.factor(mu, N, P, E)
    fac = ctx().factor(mu, N, 8, P, E, form)
    ctx().sync(fac)
    _check_factor(fac, f, N)


def test_beta1_pivots_closed_form_n128():
    # D_m = (m!)^2 exactly: every intermediate is an integer, no rounding occurs
    N, P = 128, 4096
    say("beta1 closed form", N, P)
    mu = moments(1, 2 * N - 1)
    fac = ctx().factor(mu, N, 8, P, 16, "valu")
    ctx().sync(fac)
    s = fac.s_list()
    W = 2 * P - 4
    piv = fac.pivots()
    for m in range(N):
        assert piv[m] == math.factorial(m) ** 2 << (W - 2 * s[m]), m
    h = fac.h_list()
    for i in (0, 5, 63, 100):
        got = fac.multipliers(i)
        for r, v in zip(range(i + 1, N), got):
            L = math.comb(r, i) * math.factorial(r) // math.factorial(i)
            assert v == L << (s[i] + h[i] - s[r])


def test_not_positive_definite_reports_pivot():
    from hankel_inputs import Dyadic
    from paper_1810_01478_amd._lib import HLError, HL_ENOTPD
    mu = [Dyadic(4, 0), Dyadic(4, 0), Dyadic(3, 0), Dyadic(9, 0), Dyadic(30, 0)]
    say("not PD")
    fac = ctx().factor(mu, 3, 1, 256, 1, "valu")
    with pytest.raises(HLError) as e:
        ctx().sync(fac)
    assert e.value.code == HL_ENOTPD and "index 1" in str(e.value)


def test_mfma_output_layout():
    # v_mfma_i32_32x32x32_i8: lane l, register v holds row 8(v/4) + 4(l/32) + v%4, column l%32
    say("mfma layout")
    out = ctx().debug_mfma_layout()
    for v in range(16):
        for l in range(64):
            m = 8 * (v // 4) + 4 * (l // 32) + (v % 4)
            n = l % 32
            assert out[v * 64 + l] == 32 * (m + 1), (v, l, out[v * 64 + l])
            assert out[1024 + v * 64 + l] == 32 * (n + 1), (v, l)


@pytest.mark.parametrize("beta,N,P,E", [
    (Fraction(1, 2), 64, 2048, 16),
    (Fraction(1, 2), 80, 1024, 7),
    (Fraction(1, 3), 45, 1536, 1),
    (Fraction(1, 2), 100, 4096, 16),
    (Fraction(1, 2), 70, 2176, 16),   # 2S = 544 digits: a second, partial limb range
])
def test_factor_mfma_bit_exact_vs_oracle(beta, N, P, E):
    say("factor mfma", beta, N, P, E)
    mu = moments(beta, 2 * N - 1)
    f = C.factor(mu, N, P, E)
    fac = ctx().factor(mu, N, 8, P, E, "mfma")
    ctx().sync(fac)
    _check_factor(fac, f, N)


def test_mfma_equals_valu_bitwise_c2b_shape():
    # beta = 1/2, N = 256 at 8192 bits: both forms of the update give the same bits
    N, P = 256, 8192
    say("mfma vs valu", N, P)
    mu = moments(Fraction(1, 2), 2 * N - 1)
    fa = ctx().factor(mu, N, 8, P, 16, "mfma")
    ctx().sync(fa)
    fb = ctx().factor(mu, N, 8, P, 16, "valu")
    ctx().sync(fb)
    import torch
    assert torch.equal(fa.d, fb.d) and torch.equal(fa.l, fb.l) and torch.equal(fa.h, fb.h)


@pytest.mark.parametrize("beta,N,P,E", [
    (Fraction(1, 2), 64, 2048, 16),
    (Fraction(1, 2), 80, 1024, 7),    # ragged last tile
    (Fraction(1, 3), 45, 1536, 1),
    (Fraction(1, 2), 100, 4096, 16),
    (Fraction(1, 3), 20, 256, 1),     # 32 digits split as 256 (zero digits on top)
    (1, 97, 3072, 4),
    (Fraction(1, 3), 128, 19072, 16),  # a batched-workload precision: 2384 digits split as 2560
])
@pytest.mark.parametrize("levels", [1, 2, 3, 4])
def test_factor_karatsuba_bit_exact_vs_oracle(beta, N, P, E, levels):
    # the Karatsuba forms of the trailing update are exact: same bits as the
    # oracle at every level and precision (the split digit strings are the
    # factor's S = P/8 digits with zero digits up to a multiple of 128)
    say("factor karatsuba", beta, N, P, E, levels)
    mu = moments(beta, 2 * N - 1)
    f = C.factor(mu, N, P, E)
    c = ctx()
    c.set_karatsuba(levels)
    try:
        fac = c.factor(mu, N, 8, P, E, "mfma")
        c.sync(fac)
    finally:
        c.set_karatsuba(-1)
    _check_factor(fac, f, N)


def test_karatsuba_equals_digit_product_c2b_shape():
    # beta = 1/2, N = 256 at 8192 bits: the digit product, one, two and three
    # Karatsuba levels, and a continuation in pieces that switches form between
    # pieces, all give the same bits
    import torch
    N, P = 256, 8192
    say("karatsuba vs digit product", N, P)
    mu = moments(Fraction(1, 2), 2 * N - 1)
    c = ctx()
    got = []
    try:
        c.set_karatsuba(0)
        fa = c.factor(mu, N, 8, P, 16, "mfma")
        c.sync(fa)
        for lv in (1, 2, 3, 4):
            c.set_karatsuba(lv)
            fb = c.factor(mu, N, 8, P, 16, "mfma")
            c.sync(fb)
            got.append(fb)
        fc = c.factor_cols(mu, N, 8, P, 16, "mfma", 0, 96)
        for lv, (c0, c1) in zip((0, 3, 1, 2), ((96, 128), (128, 160), (160, 208), (208, N))):
            c.set_karatsuba(lv)
            c.factor_cols(mu, N, 8, P, 16, "mfma", c0, c1, fac=fc)
        c.sync(fc)
        got.append(fc)
    finally:
        c.set_karatsuba(-1)
    for f in got:
        assert torch.equal(fa.d, f.d) and torch.equal(fa.l, f.l) and torch.equal(fa.h, f.h)


@pytest.mark.parametrize("N,P", [(200, 8320), (160, 10368)])
def test_karatsuba_padded_digits_equal_digit_product(N, P):
    # P not a multiple of 1024: the split strings carry zero digits above the
    # factors' (1040 -> 1280, 1296 -> 1536 digits); every level gives the digit
    # product's bits
    import torch
    say("karatsuba padded digits", N, P)
    mu = moments(Fraction(1, 2), 2 * N - 1)
    c = ctx()
    try:
        c.set_karatsuba(0)
        fa = c.factor(mu, N, 8, P, 16, "mfma")
        c.sync(fa)
        for lv in (1, 2, 3, 4):
            c.set_karatsuba(lv)
            fb = c.factor(mu, N, 8, P, 16, "mfma")
            c.sync(fb)
            assert torch.equal(fa.d, fb.d) and torch.equal(fa.l, fb.l) and torch.equal(fa.h, fb.h), lv
    finally:
        c.set_karatsuba(-1)


def test_set_karatsuba_rejects_bad_mode():
    from paper_1810_01478_amd._lib import HLError, HL_EINVAL
    with pytest.raises(HLError) as e:
        ctx().set_karatsuba(5)
    assert e.value.code == HL_EINVAL


def test_live_trailing_matrix_equal_across_forms():
    # after the first 96 columns (beta = 1/2, N = 256, 8192 bits) the part of the
    # trailing matrix still to be factored (tiles (R, C), C >= 3) is the same in
    # the VALU form and the MFMA form, whose pivot lookahead leaves the dead
    # diagonal entries of factored columns alone
    import torch
    N, P, cols = 256, 8192, 96
    say("live trailing matrix", N, P, cols)
    mu = moments(Fraction(1, 2), 2 * N - 1)
    c = ctx()
    fa = c.factor_cols(mu, N, 8, P, 16, "mfma", 0, cols)
    c.sync(fa)
    fb = c.factor_cols(mu, N, 8, P, 16, "valu", 0, cols)
    c.sync(fb)
    so, tb = fa.sizes.trail_offset, 1024 * 2 * (P // 32) * 4
    assert so == fb.sizes.trail_offset
    for R in range(cols // 32, N // 32):
        t0 = so + (R * (R + 1) // 2 + cols // 32) * tb
        t1 = so + (R * (R + 1) // 2 + R + 1) * tb
        assert torch.equal(fa.ws[t0:t1], fb.ws[t0:t1]), R
    assert torch.equal(fa.d[:cols * 2 * (P // 32)], fb.d[:cols * 2 * (P // 32)])
