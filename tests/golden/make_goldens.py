"""Write the oracle's records for the parity tests at the benchmark sizes.

Calls only ``oracle/`` (and ``hankel_inputs`` for the moments); nothing here
comes from the GPU library.  Each record holds, for beta = 1/2 and the given
N, k, P, E (scales of Section 6.2's preconditioner, Algorithm 1, Algorithm 4,
eq. ``equ:index``, Sections 4.2 and 4.5):

* s_j and h_i in full;
* per column i, the SHA-256 of d_i (2P/32 little-endian 32-bit limbs, two's
  complement) and of the multipliers b_ri, r = i+1 .. N-1 (P/32 limbs each);
* per column m < k of L^-1's leading columns, the SHA-256 of x_rm, r = 0 .. N-1;
* the SHA-256 of the k x k block (row-major, P/32 limbs per entry), its
  exponent, and lambda_1, lambda_1 of the (k-1) block and their difference (the
  truncation estimate) to 200 significant digits, from the eigen-solve at
  2P + 64 bits.

    python tests/golden/make_goldens.py c2b            # N = 256,  P = 8192,  k = 8
    python tests/golden/make_goldens.py n256_p32768    # N = 256,  P = 32768, k = 8
    python tests/golden/make_goldens.py c4             # N = 1024, P = 49152, k = 16
    python tests/golden/make_goldens.py c4_2p          # N = 1024, P = 98304, k = 16
"""
import argparse
import hashlib
import json
import os
import sys
import time
from fractions import Fraction

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import mpmath  # noqa: E402

from hankel_inputs import moments  # noqa: E402
from oracle import contract as C  # noqa: E402
from oracle import parallel as PAR  # noqa: E402

RECORDS = {
    "c2b": dict(N=256, k=8, P=8192, E=16),
    "n256_p32768": dict(N=256, k=8, P=32768, E=16),
    "c4": dict(N=1024, k=16, P=49152, E=16),
    "c4_2p": dict(N=1024, k=16, P=98304, E=16),
}


def path(name):
    return os.path.join(HERE, "oracle_beta_half_%s.json" % name)


def make(name, nproc):
    cfg = RECORDS[name]
    N, k, P, E = cfg["N"], cfg["k"], cfg["P"], cfg["E"]
    nl = P // 32
    mu = moments(Fraction(1, 2), 2 * N - 1)
    t0 = time.time()
    pf = PAR.factor_solve(mu, N, P, E, k, nproc)
    t1 = time.time()
    bl = PAR.block(pf, nproc)
    t2 = time.time()
    ev = C.eigen(bl, P=P)
    t3 = time.time()
    with mpmath.workprec(ev.prec):
        rec = {
            "what": "oracle record, beta = 1/2 (mu_j = 2 (2j+1)!)",
            "beta": "1/2", "N": N, "k": k, "P": P, "E": E,
            "s": pf.s, "h": pf.h,
            "d_sha256": pf.d_sha, "b_sha256": pf.b_sha,
            "x_sha256": [PAR.column_digest([pf.X[r][m] for r in range(N)], nl) for m in range(k)],
            "w_sha256": PAR.column_digest(pf.w, nl + 2),
            "blk_sha256": PAR.column_digest([v for row in bl.blk for v in row], nl),
            "blk_exp": bl.blk_exp, "tau": bl.tau,
            "lam1": mpmath.nstr(ev.lam1, 200), "lam1_km1": mpmath.nstr(ev.lam1_km1, 200),
            "trunc": mpmath.nstr(ev.trunc, 200), "eig_prec": ev.prec,
            "oracle_seconds": {"factor_solve": round(t1 - t0, 1), "block": round(t2 - t1, 1),
                               "eigen": round(t3 - t2, 1)},
            "processes": nproc,
        }
    with open(path(name), "w") as f:
        json.dump(rec, f, indent=0)
        f.write("\n")
    print(name, rec["oracle_seconds"], "lambda_1 =", rec["lam1"][:40], flush=True)


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("names", nargs="+", choices=sorted(RECORDS))
    ap.add_argument("--procs", type=int, default=os.cpu_count() or 1)
    a = ap.parse_args()
    for n in a.names:
        make(n, a.procs)
