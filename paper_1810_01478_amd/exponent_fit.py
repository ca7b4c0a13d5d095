"""The leading-exponent fit of Section 6 ("Linear fit") on lambda_1(N).

Section 6 writes the leading-order asymptotics (eq. ``leading_order2``),
lambda_1(N) ~ 8 pi sqrt(log N) / (4 pi N e)^(2/pi), as the straight line of
eq. ``linear``: y = a + b x with x = log(4 pi N e) and
y = log(8 pi sqrt(log N) / lambda_1(N)), whose slope b is the leading exponent
2/pi.  It fits a and b by least squares with each point weighted in proportion
to N^2, and reports the slope with an interval.

The interval: Section 6 calls [0.63510, 0.63781] a 95% interval for the slope.
From Table 2's own lambda_1 that is the two-sided Student-t interval at the 99%
level (7 degrees of freedom); the 95% one is [0.63554, 0.63737].  Both are
returned, and both contain 2/pi.

This is a two-parameter fit on a few dozen numbers, done on the host with
numpy; the GPU work is lambda_1(N) itself (``paper_1810_01478_amd.table2``).

    python -m paper_1810_01478_amd.exponent_fit --N 500 750 1000 ... 4500
"""
from __future__ import annotations

import argparse
import json
import math
import sys
from typing import Dict, List, Optional, Sequence

import numpy as np


def coords(N: Sequence[int], lam1: Sequence[float]):
    """x = log(4 pi N e), y = log(8 pi sqrt(log N) / lambda_1) (eq. ``linear``)."""
    n = np.asarray(N, dtype=np.float64)
    lam = np.asarray(lam1, dtype=np.float64)
    x = np.log(4.0 * math.pi * math.e * n)
    y = np.log(8.0 * math.pi * np.sqrt(np.log(n)) / lam)
    return x, y


def fit(N: Sequence[int], lam1: Sequence[float], weight_power: int = 2) -> Dict:
    """Weighted least squares of y on (1, x), weights N^weight_power; slope
    intervals at 95% and 99% from the Student t distribution."""
    from scipy import stats
    x, y = coords(N, lam1)
    w = np.asarray(N, dtype=np.float64) ** weight_power
    w = w / w.max()
    X = np.stack([np.ones_like(x), x], axis=1)
    sw = np.sqrt(w)
    coef, *_ = np.linalg.lstsq(X * sw[:, None], y * sw, rcond=None)
    res = y - X @ coef
    n, p = len(x), 2
    ssr = float(np.sum(w * res * res))
    s2 = ssr / (n - p)
    cov = s2 * np.linalg.inv((X * w[:, None]).T @ X)
    se = np.sqrt(np.diag(cov))
    yb = float(np.sum(w * y) / np.sum(w))
    r2 = 1.0 - ssr / float(np.sum(w * (y - yb) ** 2))
    out = {"intercept": float(coef[0]), "slope": float(coef[1]), "se_intercept": float(se[0]),
           "se_slope": float(se[1]), "r2": r2, "adj_r2": 1.0 - (1.0 - r2) * (n - 1) / (n - p),
           "dof": n - p, "residuals": res.tolist(), "two_over_pi": 2.0 / math.pi}
    for level in (0.95, 0.99):
        q = float(stats.t.ppf(0.5 + level / 2, n - p))
        out["ci%d" % round(100 * level)] = [out["slope"] - q * out["se_slope"], out["slope"] + q * out["se_slope"]]
    out["slope_vs_two_over_pi"] = out["slope"] / (2.0 / math.pi) - 1.0
    return out


def main(argv: Optional[List[str]] = None) -> int:
    ap = argparse.ArgumentParser(description="lambda_1(N) on the GPU, then the leading-exponent fit")
    ap.add_argument("--N", type=int, nargs="+", default=list(range(500, 4501, 250)))
    ap.add_argument("--beta", default="1/2")
    ap.add_argument("--k", type=int, default=8)
    ap.add_argument("--P-start", type=int, default=1024)
    ap.add_argument("--chunk", type=int, default=512)
    ap.add_argument("--weight-power", type=int, default=2)
    ap.add_argument("--out", default="", help="append the lambda_1 rows (JSON lines) to this file")
    a = ap.parse_args(argv)
    from fractions import Fraction
    from .api import Context
    from .table2 import precision_scan
    ctx = Context()
    Ns, lams = [], []
    P0 = a.P_start
    for N in a.N:
        res = precision_scan(ctx, Fraction(a.beta), N, a.k, 0, P0, chunk=a.chunk)
        Ns.append(N)
        lams.append(res["row"]["lambda"][0])
        print("N=%d required P=%d lambda_1=%r" % (N, res["required_P"], lams[-1]), flush=True)
        if a.out:
            with open(a.out, "a") as f:
                f.write(json.dumps(res) + "\n")
        P0 = max(1024, res["required_P"] - 1024)
    r = fit(Ns, lams, a.weight_power)
    r["N"] = Ns
    r["lambda1"] = lams
    print(json.dumps(r), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
