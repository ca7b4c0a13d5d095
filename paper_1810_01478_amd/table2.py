"""Table 2 of the paper on one GPU: the three smallest eigenvalues of H_N with
their truncation estimates, the required precision and the time per stage.

The precision scan follows the "Required Precision" column (Section 5, with
the validation rule of Section 4.1): the precision runs over P_start,
P_start + step, ...; the required precision is the first P whose eigenvalues
agree with those computed at P + step to a relative 1e-15.  A run that stops
with ENOTPD, EOVERFLOW or ENOCONV (too few bits for this N) agrees with nothing.  The
eigenvalues compared are lambda_1 .. lambda_(count+1) of the k x k block and of
its leading (k-1) x (k-1) block (the truncation estimates are their differences).

Here P is the precision of the scaled fixed-point contract (numbers of P bits
relative to their row's power-of-two scale, Section 6.2's preconditioner with
one scale per row, E = 1); the paper's K counts bits right of a single binary
point, so the two are comparable in size but are not the same quantity.

    python -m paper_1810_01478_amd.table2 --N 500 1000 1500
"""
from __future__ import annotations

import argparse
import json
import sys
import time
from fractions import Fraction
from typing import Dict, List, Optional

import torch

from . import _lib as L
from .api import Context, _moments


def _log(*a):
    print(*a, flush=True)


def run_at(ctx: Context, beta, N: int, k: int, P: int, E: int = 1, form: str = "mfma", count: int = 2,
           chunk: int = 0) -> Dict:
    """One evaluation at precision P: factor -> block -> lambda_1 .. lambda_(count+1).
    Returns the eigenvalues and per-stage seconds, or {"error": ...} when the
    precision is too small (ENOTPD, EOVERFLOW, ENOCONV).  chunk > 0 factors in pieces
    of that many columns with a progress line after each."""
    mu = _moments(beta, 2 * N - 1, mant_bits=P + 64)
    sh = ctx.shape(N, k, P, E, form)
    fac = ctx.alloc(sh)
    packed = ctx.pack_moments(mu[:2 * N - 1])
    torch.cuda.synchronize()
    ctx.set_timing(True)
    t0 = time.perf_counter()
    rec: Dict = {"N": N, "P": P, "k": k, "E": E, "form": form}
    try:
        if chunk <= 0:
            ctx.factor(mu, N, k, P, E, form, fac=fac, packed=packed)
            t_fac = ctx.timing()["ms"][7]
        else:
            t_fac = 0.0
            for c0 in range(0, N, chunk):
                c1 = min(N, c0 + chunk)
                ctx.factor_cols(mu, N, k, P, E, form, c0, c1, fac=fac, packed=packed)
                t_fac += ctx.timing()["ms"][7]
                _log("  N=%d P=%d columns %d..%d  %.1f s" % (N, P, c0, c1, time.perf_counter() - t0))
        ctx.inv_block(fac)
        t1 = ctx.timing()["ms"]
        r1 = ctx.eigen(fac, want_mant=False)
        t_eig = ctx.timing()["ms"][4]
        te = time.perf_counter()
        nxt = ctx.lambda_next(fac, count, want_mant=False) if count > 0 else []
        torch.cuda.synchronize()
        t_next = time.perf_counter() - te
    except L.HLError as e:
        if e.code not in (L.HL_ENOTPD, L.HL_EOVERFLOW, L.HL_ENOCONV):
            raise
        rec["error"] = str(e)
        rec["wall_s"] = time.perf_counter() - t0
        return rec
    finally:
        ctx.set_timing(False)
        del fac
        torch.cuda.empty_cache()
    rec["lambda"] = [r1["lambda1"]] + [g["lambda"] for g in nxt]
    rec["lambda_km1"] = [r1["lambda1_km1"]] + [g["lambda_km1"] for g in nxt]
    rec["trunc"] = [r1["trunc"]] + [g["trunc"] for g in nxt]
    rec["seconds"] = {"ldlt": t_fac / 1e3, "linv": t1[2] / 1e3, "block": t1[3] / 1e3,
                      "eigen_lambda1": t_eig / 1e3, "eigen_next": t_next}
    rec["wall_s"] = time.perf_counter() - t0
    return rec


def agree(a: Dict, b: Dict, tol: float) -> bool:
    """Both runs succeeded and every eigenvalue agrees to a relative tol."""
    if "error" in a or "error" in b:
        return False
    for key in ("lambda", "lambda_km1"):
        for x, y in zip(a[key], b[key]):
            if not abs(x / y - 1) <= tol:
                return False
    return True


def precision_scan(ctx: Context, beta, N: int, k: int = 8, count: int = 2, P_start: int = 1024,
                   step: int = 1024, tol: float = 1e-15, E: int = 1, form: str = "mfma",
                   P_max: int = 57344 - 1024, chunk: int = 0) -> Dict:
    """The required precision of Table 2 (smallest P from P_start in steps of
    `step` whose eigenvalues agree with P + step to `tol`) and the row at it."""
    runs: List[Dict] = []
    P = P_start
    prev = run_at(ctx, beta, N, k, P, E, form, count, chunk)
    runs.append(prev)
    _log(json.dumps(prev))
    while P + step <= P_max:
        cur = run_at(ctx, beta, N, k, P + step, E, form, count, chunk)
        runs.append(cur)
        _log(json.dumps(cur))
        if agree(prev, cur, tol):
            return {"N": N, "required_P": P, "row": prev, "check": cur, "runs": runs}
        prev = cur
        P += step
    raise RuntimeError("N=%d: no agreement to %g below P=%d" % (N, tol, P_max))


def main(argv: Optional[List[str]] = None) -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--N", type=int, nargs="+", default=[500, 1000, 1500, 2000, 2500, 3000, 3500, 4000, 4500])
    ap.add_argument("--beta", default="1/2")
    ap.add_argument("--k", type=int, default=8)
    ap.add_argument("--count", type=int, default=2, help="further eigenvalues beyond lambda_1 (0, 1 or 2)")
    ap.add_argument("--P-start", type=int, default=1024,
                    help="first precision of the first N; each later N starts one step below the previous result")
    ap.add_argument("--step", type=int, default=1024)
    ap.add_argument("--tol", type=float, default=1e-15)
    ap.add_argument("--E", type=int, default=1)
    ap.add_argument("--form", default="mfma", choices=["mfma", "valu"])
    ap.add_argument("--chunk", type=int, default=512, help="columns per progress line (0: one call)")
    ap.add_argument("--out", default="", help="append one JSON line per N to this file")
    a = ap.parse_args(argv)
    beta = Fraction(a.beta)
    ctx = Context()
    P0 = a.P_start
    for N in a.N:
        t0 = time.perf_counter()
        res = precision_scan(ctx, beta, N, a.k, a.count, P0, a.step, a.tol, a.E, a.form, chunk=a.chunk)
        res["scan_wall_s"] = time.perf_counter() - t0
        row = res["row"]
        _log("N=%d required P=%d lambda=%s trunc=%s ldlt=%.2f s wall=%.2f s (scan %.1f s)" % (
            N, res["required_P"], row["lambda"], row["trunc"], row["seconds"]["ldlt"], row["wall_s"],
            res["scan_wall_s"]))
        if a.out:
            with open(a.out, "a") as f:
                f.write(json.dumps(res) + "\n")
        P0 = max(a.step, res["required_P"] - a.step)
    return 0


if __name__ == "__main__":
    sys.exit(main())
