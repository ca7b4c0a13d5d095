"""Batched path (hl_batch_*): a batch of uneven instances gives, on every replay
of its captured graph, the same bits as the single-instance path (itself
bit-exact with the oracle), and the oracle's pivots and block directly for the
small instances and, for two N = 256 instances, every bit of the oracle's
records; the autotuner's choice gives the same bits."""
import math
from fractions import Fraction

import pytest
import torch

from hankel_inputs import batch_configs, moments
from oracle import contract as C

from gpu_util import ctx, say

pytestmark = pytest.mark.gpu

SPECS = [
    (Fraction(1, 2), 64, 8, 2048, 16, "mfma"),
    (Fraction(1), 40, 5, 1024, 7, "valu"),
    (Fraction(1, 3), 100, 8, 4096, 16, "mfma"),
    (Fraction(2, 3), 33, 3, 1536, 16, "mfma"),
    (Fraction(1, 2), 130, 16, 8192, 16, "mfma"),      # one Karatsuba level by default
    (Fraction(1), 17, 1, 512, 1, "valu"),
    (Fraction(1, 3), 96, 8, 17024, 16, "mfma"),       # two levels, digits padded 2128 -> 2176
    (Fraction(1, 2), 70, 8, 33024, 16, "mfma"),       # three levels, 4128 -> 4224
]


def _mu(beta, N, P):
    return moments(beta, 2 * N - 1, P + 64)


def _single(mu, N, k, P, E, form):
    fac = ctx().factor(mu, N, k, P, E, form)
    res = ctx().lambda_min(fac)
    return fac, res


def _same(fb, fs, N):
    assert fb.pivots() == fs.pivots()
    assert torch.equal(fb.l, fs.l)
    assert torch.equal(fb.x[:fs.x.numel()], fs.x)
    assert fb.block() == fs.block()


def test_batch_matches_single_instances_over_replays():
    from paper_1810_01478_amd.api import Batch
    mus = [_mu(b, N, P) for (b, N, k, P, E, f) in SPECS]
    say("batch of", len(SPECS))
    batch = Batch(ctx(), [(mu, N, k, P, E, f) for mu, (b, N, k, P, E, f) in zip(mus, SPECS)])
    singles = [_single(mu, N, k, P, E, f) for mu, (b, N, k, P, E, f) in zip(mus, SPECS)]
    for rep in range(3):
        say("replay", rep)
        batch.launch()
        res = batch.results()
        for j, ((b, N, k, P, E, f), (fs, rs)) in enumerate(zip(SPECS, singles)):
            assert res[j]["status"] == 0
            _same(batch.facs[j], fs, N)
            assert res[j]["lambda1"] == rs["lambda1"], j
            assert res[j]["trunc"] == rs["trunc"] or (math.isnan(res[j]["trunc"]) and math.isnan(rs["trunc"])), j
        # eager work on the same device between replays
        _single(mus[0], *SPECS[0][1:])
        torch.cuda.synchronize()
    # the oracle directly, for the instances it finishes quickly
    for j, (b, N, k, P, E, f) in enumerate(SPECS):
        if N > 70:
            continue
        fo, sv, bl, ev = C.lambda_min(mus[j], N, k, P, E)
        assert batch.facs[j].pivots() == fo.d, j
        blk, bexp = batch.facs[j].block()
        assert blk == bl.blk and bexp == bl.blk_exp, j
    batch.close()


def test_autotuned_batch_gives_the_same_bits():
    from paper_1810_01478_amd.api import Batch, autotune
    specs = SPECS[:4]
    mus = [_mu(b, N, P) for (b, N, k, P, E, f) in specs]
    batch = Batch(ctx(), [(mu, N, k, P, E, f) for mu, (b, N, k, P, E, f) in zip(mus, specs)])
    tune, ms = autotune(batch, panels=2)
    say("autotune", tune, "%.2f ms" % ms)
    assert tune["items_per_simd"] in (2, 4, 8) and ms > 0
    tuned = Batch(ctx(), [(mu, N, k, P, E, f) for mu, (b, N, k, P, E, f) in zip(mus, specs)], tune=tune)
    batch.launch()
    r0 = batch.results()
    tuned.launch()
    r1 = tuned.results()
    for j in range(len(specs)):
        _same(tuned.facs[j], batch.facs[j], specs[j][1])
        assert r0[j]["lambda1"] == r1[j]["lambda1"]
    batch.close()
    tuned.close()


def test_batch_update_forms_give_the_same_bits():
    # the trailing updates as the digit product (karatsuba -1) and with three
    # Karatsuba levels for every MFMA instance: the same bits as the default
    from paper_1810_01478_amd.api import Batch
    specs = [SPECS[j] for j in (0, 2, 4, 6, 7)]
    mus = [_mu(b, N, P) for (b, N, k, P, E, f) in specs]
    runs = []
    for kk in (0, -1, 3):
        say("batch karatsuba", kk)
        bt = Batch(ctx(), [(mu, N, k, P, E, f) for mu, (b, N, k, P, E, f) in zip(mus, specs)],
                   tune={"items_per_simd": 8, "range_cap": 64, "valu_below_bits": 0, "karatsuba": kk})
        bt.launch()
        runs.append((bt, bt.results()))
    (b0, r0) = runs[0]
    for bt, r in runs[1:]:
        for j in range(len(specs)):
            _same(bt.facs[j], b0.facs[j], specs[j][1])
            assert r[j]["lambda1"] == r0[j]["lambda1"]
    for bt, _r in runs:
        bt.close()


def test_batch_instances_bit_exact_vs_oracle_records():
    # the oracle's records at N = 256 (beta = 1/2, k = 8: P = 8192 with one
    # Karatsuba level, P = 32768 with three) as instances of one uneven batch:
    # every pivot, multiplier, column of L^-1 and the block bit for bit, and
    # lambda_1 from the batch's block against the record
    from paper_1810_01478_amd.api import Batch
    from test_gpu_goldens import check_factor_bits, check_solve_block, digits, record
    recs = [record("c2b"), record("n256_p32768")]
    specs = [(moments(Fraction(1, 2), 2 * r["N"] - 1), r["N"], r["k"], r["P"], r["E"], "mfma") for r in recs]
    b, N, k, P, E, f = SPECS[2]
    specs.append((_mu(b, N, P), N, k, P, E, f))
    say("batch with the N = 256 oracle records")
    batch = Batch(ctx(), specs)
    batch.launch()
    res = batch.results()
    for j, rec in enumerate(recs):
        assert res[j]["status"] == 0, j
        fac = batch.facs[j]
        check_factor_bits(fac, rec)
        check_solve_block(fac, rec)
        assert abs(res[j]["lambda1"] / float(rec["lam1"]) - 1) < 1e-14, j
        dl, dt = digits(ctx().lambda_min(fac), rec, 2 * rec["P"])
        say("  record", j, "lambda_1 digits %.0f, truncation digits %.0f" % (min(dl, 1e9), min(dt, 1e9)))
        assert dl >= 150 and dt >= 100, j
    assert res[2]["status"] == 0
    batch.close()


@pytest.mark.timeout(600)
def test_batched_workload_sampled_against_single_instances():
    # the batched workload: 64 instances, beta in {1/3, 1/2, 2/3, 1}, N in
    # [32, 512], P from the condition estimate; four instances re-run alone
    from paper_1810_01478_amd.api import Batch
    cfg = batch_configs()
    specs = [(moments(b, 2 * N - 1, P + 64), N, 8, P, 16, "mfma") for (b, N, P) in cfg]
    say("batched workload", len(specs))
    batch = Batch(ctx(), specs)
    batch.launch()
    res = batch.results()
    assert all(r["status"] == 0 for r in res)
    assert all(r["lambda1"] > 0 and r["trunc"] <= 0 for r in res)
    for j in (0, 7, 31, 63):
        mu, N, k, P, E, f = specs[j]
        say("  instance", j, cfg[j])
        fs, rs = _single(mu, N, k, P, E, f)
        _same(batch.facs[j], fs, N)
        assert res[j]["lambda1"] == rs["lambda1"]
    batch.close()
