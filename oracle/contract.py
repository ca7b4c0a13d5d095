"""The fixed-point contract, step by step, in plain Python integers.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Number format (Section 4.1, eq. ``precision``).  The paper keeps every matrix
element as an integer over 2**K and carries twice as many fractional bits through
the LDL^T.  Here the precision P plays the role of K: the trailing matrix holds
2P-bit integers, the factors hold P-bit integers, and nothing inside the O(N^3)
update is rounded.  Because the entries of H_N grow factorially along the diagonal
(Section 2, eq. ``matrix``), a single global binary point would waste the bits of
the small rows; each row j instead carries a power-of-two scale 2**s_j, shared by
a block of E consecutive rows.  This is the diagonal pre/post-conditioning the
paper proposes in Section 6.2 (preconditioner), restricted to powers of two so
that it is exact.  With E = N and all s_j equal it is the paper's plain fixed
point.

Readings where the paper is silent (each one listed in the design doc):

* rounding: rnd(x) rounds to nearest, ties away from zero; it is applied at
  exactly these points and nowhere else: the load of H, the two factor columns u
  and b of every pivot, every entry of the first k columns of L^-1, the weights
  1/d, and the final block.  The Schur update itself is exact.
* scales: t_J = max_{j in J} bitlen(mu_{2j}) over the block J of E rows and
  s_j = ceil(t_J / 2), so that |mu_{r+c}| <= sqrt(mu_2r mu_2c) < 2**(s_r + s_c)
  (positive definiteness, Section 3).
* load: a_rc = rnd(mu_{r+c} 2**(W - s_r - s_c)), W = 2P - 4, for r >= c.
* pivot balance: for pivot d_i the factor column is split by h_i = bitlen(d_i)//2
  into u_r = rnd(a_ri / 2**h_i) (the paper's A_i[j], cut to P bits) and
  b_r = rnd(u_r w_i / 2**P) (the paper's B_i[k] = A_i[k]/A_i[i], scaled), where
  w_i = rnd(2**(2 h_i + P) / d_i), the exactly rounded quotient by the whole
  pivot, is the one division per pivot (``pivot_reciprocal``).  Algorithm 1
  precomputes B_i because divisions are expensive (Section 4.3); here the
  division is done once per pivot and each entry of B_i costs one P x P-bit
  product.  Both u and b then fit in P bits.
* update: Algorithm 1 subtracts A_i[j] * B_i[k] from A_j[k] for k >= j: the
  larger index takes the scaled factor, so a_rc -= b_r u_c for r >= c > i.
* bound: |u|, |b| and every entry of X must stay below 3 * 2**(P-3), else the
  contract reports EOVERFLOW; a pivot d_i <= 0 reports ENOTPD(i).

Parity status: every function here is pinned by tests in tests/test_oracle_*.py
(closed forms at beta = 1, exact rationals for tiny N, the brute-force
characteristic polynomial, the values the paper prints in Table 2, and
agreement at doubled precision).
"""

from __future__ import annotations

from dataclasses import dataclass, field
from typing import Dict, List, Optional, Sequence, Tuple

# status codes shared in meaning (not in code) with the library
OK, EINVAL, ENOTPD, EOVERFLOW = 0, 1, 2, 3


class ContractError(Exception):
    def __init__(self, code: int, index: int = -1, what: str = ""):
        super().__init__("contract error %d at %d: %s" % (code, index, what))
        self.code = code
        self.index = index


# ---------------------------------------------------------------- rounding

def rnd_div(a: int, d: int) -> int:
    """Nearest integer to a/d (d > 0), ties away from zero."""
    if d <= 0:
        raise ValueError("rnd_div needs d > 0")
    q = (2 * abs(a) + d) // (2 * d)
    return q if a >= 0 else -q


def rnd_shift(a: int, s: int) -> int:
    """a * 2**-s: exact for s <= 0, nearest integer (ties away) for s > 0."""
    if s <= 0:
        return a << (-s)
    q = (abs(a) + (1 << (s - 1))) >> s
    return q if a >= 0 else -q


def bitlen(M: int, e: int = 0) -> int:
    """floor(log2 |M 2**e|) + 1."""
    if M == 0:
        raise ValueError("bitlen of zero")
    return abs(M).bit_length() + e


def limit(P: int) -> int:
    """Magnitude bound for every P-bit quantity of the contract."""
    return 3 << (P - 3)


# ---------------------------------------------------------------- scales / load

def scales(mu: Sequence, N: int, E: int) -> List[int]:
    """Row scale exponents s_j (power-of-two form of the preconditioner of
    Section 6.2): s_j = ceil(t_J / 2), t_J = max over the E-row block J of
    bitlen(mu_2j)."""
    t = [bitlen(mu[2 * j].M, mu[2 * j].e) for j in range(N)]
    s: List[int] = []
    for j0 in range(0, N, E):
        tJ = max(t[j0:j0 + E])
        sJ = -((-tJ) // 2)
        s.extend([sJ] * (min(N, j0 + E) - j0))
    return s


def load_entry(mu: Sequence, r: int, c: int, W: int, s: Sequence[int]) -> int:
    """One entry of the scaled Hankel matrix: a_rc = rnd(mu_{r+c} 2**(W - s_r - s_c))."""
    m = mu[r + c]
    return rnd_shift(m.M, -(m.e + W - s[r] - s[c]))


def load(mu: Sequence, N: int, P: int, s: Sequence[int]) -> List[List[int]]:
    """Lower triangle of the scaled Hankel matrix (Section 2, eq. ``matrix``):
    a_rc = rnd(mu_{r+c} 2**(W - s_r - s_c)), rows r, columns c <= r."""
    W = 2 * P - 4
    return [[load_entry(mu, r, c, W, s) for c in range(r + 1)] for r in range(N)]


def column_factors(a: int, h: int, w: int, P: int, i: int):
    """The two factor entries of row r in column i (Algorithm 1, B_i
    precomputed): u = rnd(a_ri / 2**h_i) and b = rnd(u w_i / 2**P); both must
    stay below 3 * 2**(P-3), else EOVERFLOW at column i."""
    u = rnd_shift(a, h)
    b = rnd_shift(u * w, P)
    lim = limit(P)
    if abs(u) >= lim or abs(b) >= lim:
        raise ContractError(EOVERFLOW, i, "factor exceeds P bits")
    return u, b


# ---------------------------------------------------------------- LDL^T

def pivot_reciprocal(d: int, P: int):
    """h = bitlen(d) // 2 and w = rnd(2**(2h + P) / d): the pivot's reciprocal,
    rounded once to the nearest integer (ties away from zero), by the whole d.
    Algorithm 1 forms B_i = A_i / A_i[i]; Section 4.3 precomputes it because
    divisions are expensive, so the contract divides once per pivot and keeps
    w_i (P + 1 bits) for the multipliers and the block."""
    if d <= 0:
        raise ValueError("pivot_reciprocal needs d > 0")
    h = d.bit_length() // 2
    return h, rnd_div(1 << (2 * h + P), d)


@dataclass
class Factor:
    N: int
    P: int
    E: int
    s: List[int]
    d: List[int]                  # pivots d_i (2P-bit integers)
    h: List[int]                  # pivot balance exponents h_i
    w: List[int]                  # per-pivot reciprocals w_i = rnd(2**(2h_i+P)/d_i)
    b: List[Dict[int, int]]       # b[i][r] for r > i: multipliers of column i
    u: List[Dict[int, int]] = field(default_factory=list)  # u[i][r] (kept for checks)

    @property
    def W(self) -> int:
        return 2 * self.P - 4


def factor(mu: Sequence, N: int, P: int, E: int = 16, keep_u: bool = False,
           submul=None) -> Factor:
    """Algorithm 1 (serial LDL^T, no pivoting per the footnote of Section 4.3)
    on the scaled integer matrix, with the rounding points of the contract.

    For each column i: the pivot d_i = a_ii must be positive; w_i is its rounded
    reciprocal; the column below it gives u_r and b_r (the precomputed B_i of
    Algorithm 1); then a_rc -= b_r u_c exactly for every r >= c > i.

    ``submul(x, y, z)`` may replace ``x - y * z`` (the gmp backend); by default
    Python integers are used.
    """
    if P % 32 or P < 64:
        raise ContractError(EINVAL, -1, "P must be a positive multiple of 32")
    if N < 1 or E < 1:
        raise ContractError(EINVAL, -1, "bad N or E")
    s = scales(mu, N, E)
    A = load(mu, N, P, s)
    d: List[int] = []
    h: List[int] = []
    w: List[int] = []
    B: List[Dict[int, int]] = []
    U: List[Dict[int, int]] = []
    for i in range(N):
        di = A[i][i]
        if di <= 0:
            raise ContractError(ENOTPD, i, "pivot not positive")
        hi, wi = pivot_reciprocal(di, P)
        u: Dict[int, int] = {}
        bc: Dict[int, int] = {}
        for r in range(i + 1, N):
            u[r], bc[r] = column_factors(A[r][i], hi, wi, P, i)
        # trailing update, exact: column c, rows r >= c
        for c in range(i + 1, N):
            uc = u[c]
            if uc == 0:
                continue
            for r in range(c, N):
                if submul is None:
                    A[r][c] -= bc[r] * uc
                else:
                    A[r][c] = submul(A[r][c], bc[r], uc)
        d.append(di)
        h.append(hi)
        w.append(wi)
        B.append(bc)
        if keep_u:
            U.append(u)
        # free the finished column
        for r in range(i, N):
            A[r][i] = None
    return Factor(N=N, P=P, E=E, s=s, d=d, h=h, w=w, b=B, u=U)


def D_value(f: Factor, i: int):
    """The pivot as a rational: D_i = d_i 2**(2 s_i - W)."""
    from fractions import Fraction
    ex = 2 * f.s[i] - f.W
    return Fraction(f.d[i] << ex) if ex >= 0 else Fraction(f.d[i], 1 << -ex)


def L_value(f: Factor, r: int, i: int):
    """The multiplier as a rational: L_ri = b_ri 2**(s_r - s_i - h_i)."""
    from fractions import Fraction
    ex = f.s[r] - f.s[i] - f.h[i]
    v = f.b[i][r]
    return Fraction(v << ex) if ex >= 0 else Fraction(v, 1 << -ex)


# ---------------------------------------------------------------- first k columns of L^-1

@dataclass
class Solve:
    k: int
    G: int
    Q: int
    X: List[List[int]]            # X[r][m], m < k, zero for r < m


def solve_exponents(s: Sequence[int], k: int, W: int):
    """G = max_{m<k} s_m + 64 and Q = W - G."""
    G = max(s[:k]) + 64
    return G, W - G


def solve(f: Factor, k: int) -> Solve:
    """Algorithm 4 (first N x m columns of L^-1, Section 4.4), as a forward
    substitution on the scaled factor: x_mm = 2**(Q - h_m) and, for r > m,
    x_rm = rnd(-(sum_{i=m}^{r-1} b_ri x_im) / 2**h_r), with Q = W - G and
    G = max_{m<k} s_m + 64 (head room for 1/lambda_1 up to 2**128)."""
    N, P = f.N, f.P
    if not 1 <= k <= N:
        raise ContractError(EINVAL, -1, "need 1 <= k <= N")
    G, Q = solve_exponents(f.s, k, f.W)
    X = [[0] * k for _ in range(N)]
    for m in range(k):
        X[m][m] = linv_diag(Q, f.h[m], m)
        for r in range(m + 1, N):
            acc = 0
            for i in range(m, r):
                acc += f.b[i][r] * X[i][m]
            X[r][m] = linv_entry(acc, f.h[r], P, r)
    return Solve(k=k, G=G, Q=Q, X=X)


def linv_diag(Q: int, h: int, m: int) -> int:
    """x_mm = 2**(Q - h_m) (EOVERFLOW if Q < h_m)."""
    if Q - h < 0:
        raise ContractError(EOVERFLOW, m, "Q below h_m")
    return 1 << (Q - h)


def linv_entry(acc: int, h: int, P: int, r: int) -> int:
    """x_rm = rnd(-acc / 2**h_r) for acc = sum_{i=m}^{r-1} b_ri x_im; it must
    stay below 3 * 2**(P-3), else EOVERFLOW at row r."""
    x = rnd_shift(-acc, h)
    if abs(x) >= limit(P):
        raise ContractError(EOVERFLOW, r, "L^-1 entry exceeds P bits")
    return x


# ---------------------------------------------------------------- k x k block of H^-1

@dataclass
class Block:
    k: int
    Mt: List[List[int]]           # exact sums, scale depends on (a, b)
    blk: List[List[int]]          # common-exponent block, |blk| <= 2**(P-2)
    blk_exp: int                  # (H^-1)_ab ~= blk_ab * 2**blk_exp
    tau: int


def block(f: Factor, sv: Solve) -> Block:
    """eq. ``equ:index``: (H^-1)_ab = sum_l (L^-1)_la (L^-1)_lb / D_ll, over the
    first k columns only (Section 4.5).  With the scaled quantities and the
    per-pivot reciprocals w_r = rnd(2**(2 h_r + P) / d_r) of the factorisation:
    M_ab = sum_{r >= max(a,b)} x_ra x_rb w_r exactly, and
    (H^-1)_ab = M_ab 2**(W - 2Q - P - s_a - s_b).  The entries are brought to
    the common scale 2**(2 s* - s_a - s_b) (s* = max s_a) and rounded once to at
    most P-2 bits."""
    N, k = f.N, sv.k
    Mt = [[0] * k for _ in range(k)]
    for a in range(k):
        for b2 in range(a, k):
            Mt[a][b2] = Mt[b2][a] = block_sum(sv.X, f.w, a, b2, N)
    return block_from_sums(Mt, f.s, k, f.P, f.W, sv.Q)


def block_sum(X, w: Sequence[int], a: int, b: int, N: int) -> int:
    """M_ab = sum_{r >= max(a,b)} x_ra x_rb w_r, exactly."""
    acc = 0
    for r in range(max(a, b), N):
        acc += X[r][a] * X[r][b] * w[r]
    return acc


def block_from_sums(Mt, s: Sequence[int], k: int, P: int, W: int, Q: int) -> Block:
    """The exact sums M_ab brought to the common scale 2**(2 s* - s_a - s_b)
    (s* = max_{a<k} s_a) and rounded once to at most P-2 bits; the block is
    blk 2**blk_exp."""
    sstar = max(s[:k])
    m = [[Mt[a][b2] << (2 * sstar - s[a] - s[b2]) for b2 in range(k)] for a in range(k)]
    top = max(abs(v) for row in m for v in row)
    tau = max(0, top.bit_length() - (P - 2))
    blk = [[rnd_shift(v, tau) for v in row] for row in m]
    blk_exp = W - 2 * Q - P - 2 * sstar + tau
    return Block(k=k, Mt=Mt, blk=blk, blk_exp=blk_exp, tau=tau)


# ---------------------------------------------------------------- eigen-step

@dataclass
class Lambda:
    lam1: object                  # mpmath mpf: 1 / lambda_max(k x k block)
    lam1_km1: object              # the same from the leading (k-1) x (k-1) block
    trunc: object                 # lam1 - lam1_km1 (<= 0 by interlacing)
    lmax_blk: object              # lambda_max of the integer block (no exponent)
    prec: int


def _lmax(mat: List[List[int]], prec: int):
    import mpmath
    with mpmath.workprec(prec):
        n = len(mat)
        if n == 1:
            return mpmath.mpf(mat[0][0])
        M = mpmath.matrix(n, n)
        for a in range(n):
            for b2 in range(n):
                M[a, b2] = mpmath.mpf(mat[a][b2])
        ev = mpmath.eigsy(M, eigvals_only=True)
        return max(ev[i] for i in range(n))


def eigen(blk: Block, prec: Optional[int] = None, P: Optional[int] = None) -> Lambda:
    """Section 4.2 (sketch of the algorithm) and Section 4.5: lambda_1 is taken as
    1 / lambda_max of the k x k block of H^-1, and the truncation error as the
    difference between that and the same quantity from the leading
    (k-1) x (k-1) block, trunc = lam1(k) - lam1(k-1) (<= 0 by interlacing).  The
    largest eigenvalue of the integer block comes from a dense symmetric
    eigen-solver at ``prec`` bits (default 2P + 64: the library's precision
    doubled)."""
    import mpmath
    if prec is None:
        prec = 2 * (P or 1024) + 64
    k = blk.k
    with mpmath.workprec(prec):
        lk = _lmax(blk.blk, prec)
        lam1 = mpmath.ldexp(1 / lk, -blk.blk_exp)
        if k > 1:
            lkm1 = _lmax([row[:k - 1] for row in blk.blk[:k - 1]], prec)
            lam1m = mpmath.ldexp(1 / lkm1, -blk.blk_exp)
        else:
            lam1m = mpmath.mpf("nan")
        return Lambda(lam1=lam1, lam1_km1=lam1m, trunc=lam1 - lam1m, lmax_blk=lk, prec=prec)


@dataclass
class LambdaJ:
    j: int                        # 2, 3, ...
    lam: object                   # 1 / (j-th largest eigenvalue of the k x k block)
    lam_km1: object               # the same from the leading (k-1) x (k-1) block
    trunc: object                 # lam - lam_km1 (<= 0 by interlacing)


def _eigs_desc(mat: List[List[int]], prec: int):
    import mpmath
    with mpmath.workprec(prec):
        n = len(mat)
        M = mpmath.matrix(n, n)
        for a in range(n):
            for b2 in range(n):
                M[a, b2] = mpmath.mpf(mat[a][b2])
        ev = mpmath.eigsy(M, eigvals_only=True)
        return sorted((ev[i] for i in range(n)), reverse=True)


def eigen_next(blk: Block, count: int, prec: Optional[int] = None, P: Optional[int] = None) -> List[LambdaJ]:
    """Table 2 (Section 5) prints lambda_2 and lambda_3 beside lambda_1, each
    with its truncation estimate.  As for lambda_1 (Section 4.2), the j-th
    smallest eigenvalue of H_N is taken as 1 / (j-th largest eigenvalue of the
    k x k block of H^-1), and the estimate (Section 4.5) is that minus the same
    from the leading (k-1) x (k-1) block; Cauchy interlacing of the smaller
    block in the larger makes it <= 0.  lambda_j for j = 2 .. count + 1, so the
    (k-1) block needs count + 1 eigenvalues: k >= count + 2.  All eigenvalues
    of each integer block from one dense symmetric eigen-solve at ``prec`` bits
    (default 2P + 64)."""
    import mpmath
    if prec is None:
        prec = 2 * (P or 1024) + 64
    k = blk.k
    if count < 1 or k < count + 2:
        raise ContractError(EINVAL, k, "lambda_%d with its estimate needs k >= %d" % (count + 1, count + 2))
    with mpmath.workprec(prec):
        ek = _eigs_desc(blk.blk, prec)
        ekm1 = _eigs_desc([row[:k - 1] for row in blk.blk[:k - 1]], prec)
        out = []
        for j in range(2, count + 2):
            lam = mpmath.ldexp(1 / ek[j - 1], -blk.blk_exp)
            lamm = mpmath.ldexp(1 / ekm1[j - 1], -blk.blk_exp)
            out.append(LambdaJ(j=j, lam=lam, lam_km1=lamm, trunc=lam - lamm))
        return out


def lambda_min(mu: Sequence, N: int, k: int, P: int, E: int = 16, prec: Optional[int] = None):
    """The whole path: factor -> solve -> block -> eigen."""
    f = factor(mu, N, P, E)
    sv = solve(f, k)
    bl = block(f, sv)
    return f, sv, bl, eigen(bl, prec=prec, P=P)
