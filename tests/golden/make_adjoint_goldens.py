"""Write the oracle's records of d lambda_1 / d beta at the differentiation
workload's sizes (N = 128 and 256, P = 16384 bits, k = 8, E = 16; beta = 9/20,
1/2, 11/20).

Calls only ``oracle/`` (``oracle.adjoint.grad``: dense mpmath inverse and
eigen-solve of the definition) and ``hankel_inputs`` for the inputs: the
moments and their beta-derivatives rounded to P + 64 bits, exactly what the GPU
test passes to the library.  The oracle works at `prec` bits, far above the
condition number of H_N (about 2^4000 at N = 128 and 2^8800 at N = 256), so its
lambda_1 and derivative are good to more than a thousand digits; the records
keep 100.

    python tests/golden/make_adjoint_goldens.py --N 128 --prec 8192
    python tests/golden/make_adjoint_goldens.py --N 256 --prec 20480
"""
import argparse
import json
import os
import sys
import time
from fractions import Fraction
from multiprocessing import Pool

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import mpmath  # noqa: E402

from hankel_inputs import dmoments_dbeta, moments  # noqa: E402
from oracle import adjoint as A  # noqa: E402

BETAS = [Fraction(9, 20), Fraction(1, 2), Fraction(11, 20)]


def one(args):
    beta, N, k, P, prec = args
    t0 = time.time()
    mu = moments(beta, 2 * N - 1, P + 64)
    dmu = dmoments_dbeta(beta, 2 * N - 1, P + 64)
    t1 = time.time()
    g = A.grad(mu, dmu, N, k, prec)
    t2 = time.time()
    with mpmath.workprec(prec):
        return {"beta": "%d/%d" % (beta.numerator, beta.denominator), "N": N, "k": k, "P": P, "E": 16,
                "inputs_rounded_to_bits": P + 64, "oracle_prec": prec,
                "lam1": mpmath.nstr(g.lam1, 100), "dlam1_dbeta": mpmath.nstr(g.dlam, 100),
                "seconds": {"inputs": round(t1 - t0, 1), "oracle": round(t2 - t1, 1)}}


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("--prec", type=int, default=8192)
    ap.add_argument("--N", type=int, default=128)
    a = ap.parse_args()
    jobs = [(b, a.N, 8, 16384, a.prec) for b in BETAS]
    with Pool(len(jobs)) as pool:
        recs = pool.map(one, jobs)
    path = os.path.join(HERE, "oracle_adjoint_n%d_p16384.json" % a.N)
    with open(path, "w") as f:
        json.dump({"what": "oracle d lambda_1 / d beta (oracle.adjoint.grad)", "records": recs}, f, indent=1)
        f.write("\n")
    for r in recs:
        print(r["beta"], r["seconds"], r["dlam1_dbeta"][:40], flush=True)
