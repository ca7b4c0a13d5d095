"""Seeded pivots for the reciprocal w = rnd(2^(2h+P) / d), h = bitlen(d) // 2,
including pivots whose exact quotient lies within 2^-60 of a rounding tie
(half-integer).  Input generation only: no arithmetic of the method here."""
import random


def near_tie_pivots(P: int, count: int, seed: int):
    """Pivots d of bitlen in [P + 70, 2P - 4] (so that a cut of d to its top
    P + 64 bits drops at least six bits) with 2^e / d within about 2^-(bitlen - P - 1)
    of a half-integer, e = 2 (bitlen // 2) + P.  For an odd t, d = floor(2^(e+1)/t)
    puts the quotient just above t/2 and d + 1 just below it."""
    rng = random.Random(seed)
    out = []
    while len(out) < count:
        L = rng.randrange(P + 70, 2 * P - 3)
        e = 2 * (L // 2) + P
        # t in (2^(e+1-L), 2^(e+2-L)] gives d = 2^(e+1)/t in [2^(L-1), 2^L)
        lo, hi = 1 << (e + 1 - L), 1 << (e + 2 - L)
        t = rng.randrange(lo + 1, hi) | 1
        d0 = (1 << (e + 1)) // t
        for d in (d0, d0 + 1):
            if d.bit_length() == L:
                out.append(d)
    return out[:count]


def random_pivots(P: int, count: int, seed: int):
    """Pivots of random bit length in [2, 2P - 4] (top bit set)."""
    rng = random.Random(seed)
    out = []
    for _ in range(count):
        bits = rng.randrange(2, 2 * P - 3)
        out.append(rng.getrandbits(bits) | (1 << (bits - 1)))
    return out
