"""Parity at the benchmark sizes against the oracle's own records.

The records (tests/golden/oracle_beta_half_*.json) are written by
tests/golden/make_goldens.py, which calls only oracle/ (the row-parallel
contract on GMP); nothing in them comes from the GPU.  beta = 1/2
(mu_j = 2 (2j+1)!), E = 16:

* N = 256, P = 8192, k = 8: every Schur-update form (VALU, int8 digit product,
  one to three Karatsuba levels);
* N = 256, P = 32768, k = 8: the default form (three Karatsuba levels) and the
  VALU form;
* N = 1024, P = 49152, k = 16 (the bench workload, default form and launch
  configuration): every column's d_i and b_ri, h_i, s_j, L^-1's k leading
  columns and the block, bit for bit, and lambda_1 and the truncation estimate
  against the oracle at 2P = 98304 bits (the paper validates a precision by
  recomputing with more bits, Section 4.1; Table 2 follows that rule; the
  library itself stops at P = 57344, where the pivot's scratch fills the LDS).

Bit-exactness is checked through SHA-256 digests of the limb bytes (P/32
little-endian 32-bit limbs per multiplier, two's complement; 2P/32 per pivot).
lambda_1 must agree to at least 30 digits (the target), and here is asserted to
150 (the records keep 200)."""
import hashlib
import json
import os
from fractions import Fraction

import mpmath
import pytest

from hankel_inputs import moments

from gpu_util import ctx, say

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))


def record(name):
    p = os.path.join(HERE, "golden", "oracle_beta_half_%s.json" % name)
    if not os.path.exists(p):
        pytest.skip("oracle record %s not written yet (tests/golden/make_goldens.py %s)" % (name, name))
    with open(p) as f:
        return json.load(f)


def sha(t):
    return hashlib.sha256(t.cpu().numpy().tobytes()).hexdigest()


def check_factor_bits(fac, rec):
    N, k, nl = rec["N"], rec["k"], rec["P"] // 32
    assert fac.s_list() == rec["s"]
    assert fac.h_list() == rec["h"]
    d = fac.d.view(-1)[:N * 2 * nl].view(N, 2 * nl).cpu().numpy()
    bad_d = [i for i in range(N) if hashlib.sha256(d[i].tobytes()).hexdigest() != rec["d_sha256"][i]]
    assert not bad_d, "pivots differ at columns %s" % bad_d[:10]
    NT = fac.NT
    lv = fac.l.view(-1)
    bad_b = []
    for i in range(N - 1):
        col = lv[(i * NT + i + 1) * nl:(i * NT + N) * nl]
        if sha(col) != rec["b_sha256"][i]:
            bad_b.append(i)
    assert not bad_b, "multipliers differ in columns %s" % bad_b[:10]


def check_solve_block(fac, rec):
    N, k, nl = rec["N"], rec["k"], rec["P"] // 32
    x = fac.x.view(-1)[:N * k * nl].view(N, k, nl)
    for m in range(k):
        assert sha(x[:, m, :].contiguous()) == rec["x_sha256"][m], "L^-1 column %d" % m
    assert sha(fac.blk.view(-1)[:k * k * nl]) == rec["blk_sha256"]
    assert int(fac.blk_exp.cpu().item()) == rec["blk_exp"]


def digits(res, rec, prec):
    """Agreement of the GPU's lambda_1 and truncation estimate with a record,
    in decimal digits."""
    with mpmath.workprec(prec):
        lam = mpmath.ldexp(mpmath.mpf(res["mant"]), res["exp"])
        lamm = mpmath.ldexp(mpmath.mpf(res["mant_km1"]), res["exp_km1"])
        ref = mpmath.mpf(rec["lam1"])
        ref_t = mpmath.mpf(rec["trunc"])
        e1 = abs(lam / ref - 1)
        e2 = abs((lam - lamm) / ref_t - 1)
        f = lambda e: float("inf") if e == 0 else -float(mpmath.log10(e))
        return f(e1), f(e2)


def _run(name, forms):
    rec = record(name)
    N, k, P, E = rec["N"], rec["k"], rec["P"], rec["E"]
    c = ctx()
    mu = moments(Fraction(1, 2), 2 * N - 1)
    for form, level in forms:
        say("oracle record", name, "form", form, "karatsuba", level)
        try:
            c.set_karatsuba(level)
            fac = c.factor(mu, N, k, P, E, form)
            res = c.lambda_min(fac)
        finally:
            c.set_karatsuba(-1)
        check_factor_bits(fac, rec)
        check_solve_block(fac, rec)
        dl, dt = digits(res, rec, 2 * P)
        say("  lambda_1 digits %.0f, truncation digits %.0f" % (min(dl, 1e9), min(dt, 1e9)))
        assert dl >= 150 and dt >= 100
        del fac


def test_c2b_every_form_bit_exact():
    _run("c2b", [("valu", -1), ("mfma", 0), ("mfma", 1), ("mfma", 2), ("mfma", 3)])


def test_n256_p32768_bit_exact():
    _run("n256_p32768", [("mfma", -1), ("valu", -1)])


def _c4_gpu(rec):
    N, k, P, E = rec["N"], rec["k"], rec["P"], rec["E"]
    c = ctx()
    mu = moments(Fraction(1, 2), 2 * N - 1)
    say("C4 factor at", P, "bits, default form")
    fac = c.factor(mu, N, k, P, E, "mfma")
    res = c.lambda_min(fac)
    return fac, res


def test_c4_bit_exact():
    import torch
    rec = record("c4")
    fac, res = _c4_gpu(rec)
    check_factor_bits(fac, rec)
    check_solve_block(fac, rec)
    dl, dt = digits(res, rec, 2 * rec["P"])
    say("  vs oracle at P: lambda_1 digits %.0f, truncation digits %.0f" % (min(dl, 1e9), min(dt, 1e9)))
    assert dl >= 150 and dt >= 100
    del fac
    torch.cuda.empty_cache()


def test_c4_lambda_vs_oracle_at_doubled_precision():
    """Validate by more bits: lambda_1 and the truncation estimate from the GPU
    at P = 49152 against the oracle's at 2P = 98304."""
    import torch
    rec = record("c4")
    rec2 = record("c4_2p")
    fac, res = _c4_gpu(rec)
    dl2, dt2 = digits(res, rec2, 2 * rec2["P"])
    say("  vs oracle at 2P: lambda_1 digits %.0f, truncation digits %.0f" % (min(dl2, 1e9), min(dt2, 1e9)))
    assert dl2 >= 150 and dt2 >= 100
    del fac
    torch.cuda.empty_cache()
