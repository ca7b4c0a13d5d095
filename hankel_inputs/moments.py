"""Moment sequences of the weight w(x) = exp(-x**beta) on [0, inf).

Section 2, eq. ``moments``: mu_k = Gamma((k+1)/beta) / beta.  The Hankel matrix
of Section 2, eq. ``matrix``, is H_N = (mu_{i+j}), i, j = 0..N-1, so it needs
mu_0 .. mu_{2N-2}.

Every moment is handed over as a *dyadic* number M * 2**e (Python ints), which is
the form both the oracle and the GPU library take as input:

* beta = 1/q (q = 1, 2, 3, ...): mu_k = q * (q(k+1) - 1)!  -- exact integers
  (beta = 1 gives k!, beta = 1/2 gives 2 (2k+1)!, beta = 1/3 gives 3 (3k+2)!).
* beta = 2/q (q odd): Gamma of an integer (exact dyadic, denominator 2) or of a
  half-integer, Gamma(n + 1/2) = (2n)! sqrt(pi) / (4**n n!), whose sqrt(pi) is
  irrational; that factor is evaluated with mpmath and the product rounded to
  ``mant_bits`` significant bits.
* any other rational beta = p/q: Gamma((k+1) q / p) from p base values by
  the recurrence Gamma(x + q) = Gamma(x) * x (x+1) ... (x+q-1), rounded to
  ``mant_bits`` bits.

The derivative d mu_k / d beta = -(mu_k / beta) (1 + x psi(x)), x = (k+1)/beta,
uses psi(x + 1) = psi(x) + 1/x in the same way.

Nothing here scales, factors or rounds matrix entries: that is the method, which
the oracle and the library implement separately.
"""

from __future__ import annotations

import math
from dataclasses import dataclass
from fractions import Fraction
from typing import List, Sequence, Tuple

import numpy as np


@dataclass(frozen=True)
class Dyadic:
    """The number M * 2**e with integer M (sign in M) and integer e."""

    M: int
    e: int

    def to_fraction(self) -> Fraction:
        if self.e >= 0:
            return Fraction(self.M << self.e)
        return Fraction(self.M, 1 << (-self.e))

    def bitlen(self) -> int:
        """floor(log2 |x|) + 1 for x != 0 (the position of the top bit)."""
        if self.M == 0:
            raise ValueError("bitlen of zero")
        return abs(self.M).bit_length() + self.e

    def __float__(self) -> float:
        return float(self.to_fraction())


def _as_fraction(beta) -> Fraction:
    if isinstance(beta, Fraction):
        return beta
    if isinstance(beta, int):
        return Fraction(beta)
    # floats such as 0.45 are taken as the decimal the user wrote, exactly; a
    # decimal whose reduced denominator exceeds 10**6 is refused rather than
    # snapped to a nearby rational (pass a Fraction for such a beta)
    f = Fraction(str(beta))
    if f.denominator > 10**6:
        raise ValueError("beta = %r: its decimal %s has a denominator above 10**6; pass a Fraction" % (beta, f))
    return f


def is_exact_beta(beta) -> bool:
    """True when every moment is an exact dyadic (no irrational factor)."""
    b = _as_fraction(beta)
    return b.numerator == 1


def _round_mpf(x, mant_bits: int) -> Dyadic:
    """Round a positive or negative mpmath number to ``mant_bits`` bits."""
    import mpmath

    x = mpmath.mpf(x)
    if x == 0:
        return Dyadic(0, 0)
    sign, man, exp, bc = x._mpf_
    man = int(man)
    shift = bc - mant_bits
    if shift > 0:
        man = (man + (1 << (shift - 1))) >> shift
        exp += shift
    return Dyadic(-man if sign else man, int(exp))


def _gamma_rational(a: int, b: int, cache: dict):
    """Gamma(a / b) for integers a, b >= 1 at the current mpmath precision:
    Gamma(n + r/b) = Gamma(r/b) (r/b)(r/b + 1)...(r/b + n - 1), with
    Gamma(r/b) from the reflection formula when r/b > 1/2 and its partner is
    known."""
    import mpmath

    n, r = divmod(a, b)
    if r == 0:
        return mpmath.mpf(math.factorial(n - 1))
    g = cache.get(r)
    if g is None:
        partner = cache.get(b - r)
        if partner is not None:
            g = mpmath.pi / (mpmath.sin(mpmath.pi * r / b) * partner)
        else:
            g = mpmath.gamma(mpmath.mpf(r) / b)
        cache[r] = g
    x = mpmath.mpf(r) / b
    for j in range(n):
        g = g * (x + j)
    return g


def _digamma_rational(a: int, b: int):
    """psi(a / b) for integers a, b >= 1 at the current mpmath precision.  For
    b <= 64, Gauss's digamma theorem at the fractional part r/b (0 < r < b),
      psi(r/b) = -gamma - ln(2b) - (pi/2) cot(pi r/b)
                 + 2 sum_{n=1}^{ceil(b/2)-1} cos(2 pi n r/b) ln sin(pi n/b),
    psi(1) = -gamma, then psi(x + 1) = psi(x) + 1/x; larger b directly."""
    import mpmath

    if b > 64:
        return mpmath.digamma(mpmath.mpf(a) / b)
    n, r = divmod(a, b)
    if r == 0:
        n, r = n - 1, b
    if r == b:
        s = -mpmath.euler
    else:
        s = -mpmath.euler - mpmath.log(2 * b) - mpmath.pi / 2 * mpmath.cot(mpmath.pi * r / b)
        for j in range(1, (b + 1) // 2):
            s += 2 * mpmath.cos(2 * mpmath.pi * j * r / b) * mpmath.log(mpmath.sin(mpmath.pi * j / b))
    x = mpmath.mpf(r) / b
    for j in range(n):
        s += 1 / (x + j)
    return s


def exact_moment_fraction(beta, k: int) -> Fraction:
    """mu_k as an exact rational, for beta = 1/q or beta = 2/q at integer Gamma."""
    b = _as_fraction(beta)
    x = Fraction(k + 1) / b
    if x.denominator != 1:
        raise ValueError("moment is not rational for this beta and k")
    return Fraction(math.factorial(int(x) - 1)) / b


def moments(beta, count: int, mant_bits: int = 0) -> List[Dyadic]:
    """mu_0 .. mu_{count-1} as dyadics.

    ``mant_bits`` is the number of significant bits kept where a moment is
    irrational; exact moments are returned exactly whatever it is.
    """
    b = _as_fraction(beta)
    p, q = b.numerator, b.denominator
    out: List[Dyadic] = []
    if p == 1:
        # Gamma(q (k+1)) = (q(k+1) - 1)!, mu_k = q * that
        f = 1
        n = 0  # f = n!
        for k in range(count):
            target = q * (k + 1) - 1
            while n < target:
                n += 1
                f *= n
            out.append(Dyadic(q * f, 0))
        return out
    if mant_bits <= 0:
        raise ValueError("beta = %s has irrational moments: give mant_bits" % b)
    import mpmath

    old = mpmath.mp.prec
    try:
        mpmath.mp.prec = mant_bits + 64
        if p == 2:
            sqrt_pi = mpmath.sqrt(mpmath.pi)
            for k in range(count):
                x2 = q * (k + 1)  # x = x2 / 2
                if x2 % 2 == 0:
                    g = Fraction(math.factorial(x2 // 2 - 1))
                    val = g * Fraction(q, 2)  # mu = Gamma(x) / beta = Gamma(x) q / 2
                    num, den = val.numerator, val.denominator
                    e = 0
                    while den % 2 == 0:
                        den //= 2
                        e -= 1
                    assert den == 1
                    out.append(Dyadic(num, e))
                else:
                    n = (x2 - 1) // 2  # x = n + 1/2
                    rat = Fraction(math.factorial(2 * n), 4**n * math.factorial(n)) * Fraction(q, 2)
                    val = mpmath.mpf(rat.numerator) / rat.denominator * sqrt_pi
                    out.append(_round_mpf(val, mant_bits))
            return out
        # general rational beta = p/q: x_k = q (k+1) / p, x_{k+p} = x_k + q
        cache: dict = {}
        base = [_gamma_rational(q * (k + 1), p, cache) for k in range(min(p, count))]
        vals = list(base)
        for k in range(p, count):
            x = mpmath.mpf(q * (k + 1 - p)) / p
            g = vals[k - p]
            for j in range(q):
                g = g * (x + j)
            vals.append(g)
        inv_beta = mpmath.mpf(q) / p
        for k in range(count):
            out.append(_round_mpf(vals[k] * inv_beta, mant_bits))
        return out
    finally:
        mpmath.mp.prec = old


def dmoments_dbeta(beta, count: int, mant_bits: int) -> List[Dyadic]:
    """d mu_k / d beta = -(mu_k / beta) (1 + x psi(x)), x = (k+1)/beta."""
    import mpmath

    b = _as_fraction(beta)
    p, q = b.numerator, b.denominator
    old = mpmath.mp.prec
    try:
        mpmath.mp.prec = mant_bits + 64
        xs = [mpmath.mpf(q * (k + 1)) / p for k in range(count)]
        cache: dict = {}
        gam = [_gamma_rational(q * (k + 1), p, cache) for k in range(min(p, count))]
        psi = [_digamma_rational(q * (k + 1), p) for k in range(min(p, count))]
        for k in range(p, count):
            x = xs[k - p]
            g, s = gam[k - p], psi[k - p]
            for j in range(q):
                g = g * (x + j)
                s = s + 1 / (x + j)
            gam.append(g)
            psi.append(s)
        bet = mpmath.mpf(p) / q
        out = []
        for k in range(count):
            mu = gam[k] / bet
            out.append(_round_mpf(-(mu / bet) * (1 + xs[k] * psi[k]), mant_bits))
        return out
    finally:
        mpmath.mp.prec = old


def trace_log2(beta, N: int) -> float:
    """log2 tr(H_N) = log2 sum_{k<N} mu_{2k} (Section 2.1), via lgamma."""
    b = float(_as_fraction(beta))
    logs = [math.lgamma((2 * k + 1) / b) - math.log(b) for k in range(N)]
    m = max(logs)
    return (m + math.log(sum(math.exp(v - m) for v in logs))) / math.log(2)


def precision_rule(beta, N: int, margin: int = 512, granule: int = 128) -> int:
    """Bits of precision for one instance of the batched workload.

    Section 2.1 bounds the largest eigenvalue by the trace and takes the
    smallest to be about 1/10, so log2 cond(H_N) is estimated as
    log2 tr(H_N) + log2 10.  The precision is that estimate plus ``margin``
    bits, rounded up to a multiple of ``granule`` (the library stores numbers
    in whole 128-bit groups).
    """
    est = math.ceil(trace_log2(beta, N) + math.log2(10.0))
    bits = est + margin
    return granule * ((bits + granule - 1) // granule)


def batch_configs(count: int = 64, seed: int = 1810,
                  betas: Sequence = (Fraction(1, 3), Fraction(1, 2), Fraction(2, 3), Fraction(1)),
                  n_lo: int = 32, n_hi: int = 512) -> List[Tuple[Fraction, int, int]]:
    """The batched workload: (beta, N, P) per instance, from a seeded generator."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        bi = int(rng.integers(0, len(betas)))
        N = int(rng.integers(n_lo, n_hi + 1))
        beta = _as_fraction(betas[bi])
        out.append((beta, N, precision_rule(beta, N)))
    return out


def pack_limbs(values: Sequence[int], limbs: int) -> np.ndarray:
    """Little-endian uint32 limbs of non-negative ints, shape (len, limbs)."""
    out = np.zeros((len(values), limbs), dtype=np.uint32)
    for i, v in enumerate(values):
        if v < 0:
            raise ValueError("pack_limbs takes non-negative integers")
        if v.bit_length() > 32 * limbs:
            raise ValueError("value does not fit in %d limbs" % limbs)
        raw = v.to_bytes(4 * limbs, "little")
        out[i] = np.frombuffer(raw, dtype="<u4")
    return out


def unpack_limbs(arr: np.ndarray, signed: bool = False) -> List[int]:
    """Inverse of pack_limbs; with ``signed`` the limbs are two's complement."""
    arr = np.ascontiguousarray(arr, dtype=np.uint32)
    if arr.ndim == 1:
        arr = arr[None, :]
    out = []
    for row in arr:
        v = int.from_bytes(row.astype("<u4").tobytes(), "little")
        if signed and row.size and (int(row[-1]) >> 31):
            v -= 1 << (32 * row.size)
        out.append(v)
    return out
