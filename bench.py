"""Benchmark of the hot path on one MI355X.

A step is one pass of the whole path on one instance: moments resident in HBM
-> hl_factor (extreme-precision LDL^T of H_N) -> hl_inv_block (first k columns of
L^-1, k x k block of H^-1) -> hl_lambda_min (lambda_1 and truncation estimate),
i.e. time-to-lambda_1.

Default workload: beta = 1/2, N = 1024, k = 16, P = 49152 bits, E = 16, Schur
update as exact int8 MFMA GEMMs.  Prints one JSON line:
  value        algorithmic Schur limb-MACs of the step / step time (whole job)
  ms_per_step  time-to-lambda_1
  roofline     the int8 MFMA GEMM kernel against the int8 dense MFMA peak
  roofline_valu the plain vector-ALU form's Schur update (first two panels of
               the same matrix) against the VALU integer multiply-add peak,
               with the issue rate an ALU probe measures beside it
  cpu_baseline the CPU oracle (row-parallel contract on GMP, one process per
               host core up to 16) on the first pivots of the same matrix at
               the same precision, also a bit-exact check of those columns
  valu_sample  the plain vector-ALU form on the first two panels of the same
               matrix, checked bit-identical against the MFMA form
  adjoint      d lambda_1 / d beta on the same factorisation (hl_lambda_grad)
               and its time
  batch        the batched workload (64 uneven instances, one hipGraph replay)
"""
import argparse
import json
import math
import os
import sys
import time
from fractions import Fraction

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "limb-MAC/s in Schur update + time-to-λ₁ at N=1024 β=½ (MFMA-slice vs VALU)"

WORKLOADS = {
    # name: (beta, N, k, P, E)
    "c4": (Fraction(1, 2), 1024, 16, 49152, 16),
    "c2b": (Fraction(1, 2), 256, 8, 8192, 16),
    "c1": (Fraction(1, 2), 64, 8, 2048, 16),
    "n512": (Fraction(1, 2), 512, 8, 16384, 16),
}

MFMA_INT8_PEAK_TOPS = 5000.0      # dense int8 MFMA, MI355X: 5.0 POP/s
# vector-ALU 32 x 32 -> 64-bit integer multiply-add (v_mad_u64_u32, the plain
# form's limb product): 256 CUs x 4 SIMDs x 16 lanes, one per lane and clock
# (the issue-rate probe measures about 80% of this at the clock the GPU holds), at
# 2.4 GHz
VALU_MAD_PEAK = 256 * 4 * 16 * 2.4e9


def schur_limb_macs(N, nl):
    """Algorithmic limb multiply-adds of the whole Schur update: for every pivot
    i and every r >= c > i one P x P-bit product, nl^2 limb products each."""
    return (N - 1) * N * (N + 1) / 6 * nl * nl


def measured_traffic(workload, kernel="k_upd_mfma"):
    """HBM traffic per trailing-update launch from the rocprofv3 counter runs
    recorded under profiles/, if they were taken on this workload and on the
    kernel sources (the tile loop and its constants) as they are now; else
    None."""
    import hashlib
    path = os.path.join(ROOT, "profiles", kernel + "_c4_traffic.json")
    try:
        rec = json.load(open(path))
        for name, digest in rec["sources"].items():
            if hashlib.sha256(open(os.path.join(ROOT, name), "rb").read()).hexdigest() != digest:
                return None
    except (OSError, ValueError, KeyError, AttributeError):
        return None
    if rec.get("workload") != workload:
        return None
    return float(rec["bytes_per_launch"])


def cpu_workers():
    """Host threads for the oracle sample: the cores this process may use, at
    most 16."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def cpu_sample(mu, N, k, P, E, cols, procs):
    """The oracle (row-parallel contract on GMP, one process per core) on the
    first `cols` pivots of the same matrix: their d_i, h_i and multiplier
    columns are exactly those of the full factorisation.  Returns the oracle's
    record and the wall time of its column loop (the load of the matrix
    excluded)."""
    from oracle import parallel as PAR
    f = PAR.factor_solve(mu, N, P, E, k, procs, columns=cols)
    return f, f.column_seconds


def sample_limb_macs(N, cols, nl):
    """Schur limb multiply-adds of the first `cols` pivots of an N x N
    factorisation: pivot i updates the (N-i-1)(N-i)/2 entries r >= c > i."""
    return sum((N - i - 1) * (N - i) / 2 for i in range(cols)) * nl * nl


def kara_digit_pairs(S, levels):
    """Digit pairs one entry-column update multiplies: S^2 for the digit
    product, else the sum over the 3^L products of their operand lengths
    squared (lo halves reset the extra digits, hi halves keep them, mid halves
    add one)."""
    if levels <= 0:
        return S * S
    Sp = (S + 255) // 256 * 256
    total = 0
    for p in range(3 ** levels):
        e, div = 0, 3 ** (levels - 1)
        for _ in range(levels):
            c = (p // div) % 3
            e = 0 if c == 0 else (e if c == 1 else e + 1)
            div //= 3
        total += ((Sp >> levels) + e) ** 2
    return total


def valu_roofline(ctx, achieved, what):
    """The VALU form's Schur update against the vector ALU's integer
    multiply-add peak, with the rate the issue-rate probe measures beside it."""
    probe, _ = ctx.debug_valu_peak(mode=1)
    pair, _ = ctx.debug_valu_peak(mode=0)
    return {"bound": "alu", "achieved": achieved, "peak": VALU_MAD_PEAK, "unit": "limb-MAC/s",
            "frac": achieved / VALU_MAD_PEAK, "traffic": None, "kernel": what,
            "probe_mad_per_s": probe, "probe_mad_carry_pair_per_s": pair,
            "frac_of_probe": achieved / probe}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c4", choices=sorted(WORKLOADS))
    ap.add_argument("--form", default="mfma", choices=["mfma", "valu"])
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle sample")
    ap.add_argument("--no-valu", action="store_true", help="skip the VALU comparison sample")
    ap.add_argument("--no-grad", action="store_true", help="skip the adjoint (d lambda_1 / d beta)")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched 64-instance workload")
    ap.add_argument("--karatsuba", default="auto", choices=["auto", "0", "1", "2", "3", "4"],
                    help="Schur-update form of the MFMA path: Karatsuba levels (0: the plain digit product)")
    ap.add_argument("--cpu-cols", type=int, default=4,
                    help="pivots of the oracle sample (about 5 s each on 8 cores at the default workload)")
    ap.add_argument("--progress", action="store_true",
                    help="factor in pieces of 128 columns, printing a line after each (profiler runs)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only copy 1 GiB device to device three times (calibrates HBM byte counters) and exit")
    a = ap.parse_args()
    if a.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path (asked for --gpus %d)" % a.gpus,
              file=sys.stderr)
        sys.exit(2)

    import torch
    if a.copy_probe:
        n = 1 << 30
        x = torch.ones(n, dtype=torch.uint8, device="cuda")
        y = torch.empty_like(x)
        torch.cuda.synchronize()
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes_read": n, "copy_probe_bytes_written": n, "launches": 3}), flush=True)
        return
    from hankel_inputs import moments
    from paper_1810_01478_amd.api import Context

    beta, N, k, P, E = WORKLOADS[a.workload]
    nl = P // 32
    log = lambda *x: print("[bench]", *x, file=sys.stderr, flush=True)
    ctx = Context(0)
    ctx.set_karatsuba(-1 if a.karatsuba == "auto" else int(a.karatsuba))
    mu = moments(beta, 2 * N - 1)
    packed = ctx.pack_moments(mu)
    sh = ctx.shape(N, k, P, E, a.form)
    fac = ctx.alloc(sh)
    torch.cuda.synchronize()

    def step(timed_stages):
        """One pass of the path.  With --progress the factorisation runs in
        pieces of 128 columns with a line after each (for profiler runs, which
        serialise every launch); the per-stage times are then summed."""
        if not a.progress:
            ctx.factor(mu, N, k, P, E, a.form, fac=fac, packed=packed)
            r = ctx.lambda_min(fac)
            return r, (ctx.timing() if timed_stages else None)
        acc = None
        for c0 in range(0, N, 128):
            c1 = min(N, c0 + 128)
            ctx.factor_cols(mu, N, k, P, E, a.form, c0, c1, fac=fac, packed=packed)
            if timed_stages:
                t = ctx.timing()
                if acc is None:
                    acc = t
                else:
                    acc["ms"] = [x + y for x, y in zip(acc["ms"], t["ms"])]
                    acc["launches"] = [x + y for x, y in zip(acc["launches"], t["launches"])]
                    acc["schur_limb_macs"] += t["schur_limb_macs"]
            log("columns", c0, c1)
        r = ctx.lambda_min(fac)
        if timed_stages:
            t = ctx.timing()
            for i in (2, 3, 4):
                acc["ms"][i] = t["ms"][i]
        log("lambda_min done")
        return r, acc

    # warm-up steps; the first one with per-stage timing
    stages = None
    res = None
    for w in range(max(1, a.warmup)):
        ctx.set_timing(w == 0)
        log("warmup step", w)
        res, t = step(w == 0)
        if w == 0:
            stages = t
        ctx.set_timing(False)
    torch.cuda.synchronize()

    # timed steps
    log("timed steps", a.steps)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(a.steps):
        res, _t = step(False)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / a.steps
    macs = schur_limb_macs(N, nl)

    ms = stages["ms"]
    workload = "beta=%s N=%d k=%d P=%d E=%d form=%s" % (beta, N, k, P, E, a.form)
    out = {
        "metric": METRIC,
        "value": macs / dt,
        "unit": "limb-MAC/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": dt * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "i8" if a.form == "mfma" else "u32",
        "data": "synthetic: exact moments mu_j = Gamma((j+1)/beta)/beta generated on the host",
        "config": {"workload": workload,
                   "beta": str(beta), "N": N, "k": k, "prec_bits": P, "exp_block": E, "form": a.form},
        "time_to_lambda1_s": dt,
        "lambda1": res["lambda1"],
        "trunc": res["trunc"],
        "stages_ms": {"schur": ms[0], "mfma_gemm": ms[6], "panel": ms[1], "load": ms[5], "trsm": ms[2],
                      "block": ms[3], "eigen": ms[4], "factor_total": ms[7]},
        "schur": {"limb_macs_algorithmic": macs, "limb_macs_in_updates": stages["schur_limb_macs"],
                  "kernel_limb_mac_per_s": stages["schur_limb_macs"] / (ms[0] * 1e-3) if ms[0] else None},
    }
    lv = 0
    if a.form == "mfma" and stages["launches"][2] > 0:
        lv = round(stages["launches"][3] / stages["launches"][2])
    kara = lv > 0
    if a.form == "mfma":
        out["config"]["schur_form"] = "karatsuba x%d" % lv if kara else "digit product"
    if kara:
        out["stages_ms"]["kara_combine"] = ms[9]
    if a.form == "mfma" and ms[6] > 0:
        # int8 ops the GEMMs need per entry and panel column: the digit product
        # multiplies S^2 digit pairs (S = P/8, 16 per limb-MAC); L Karatsuba
        # levels multiply, for each of the 3^L products, its own operand length
        # squared: S'/2^L digits plus one per mid half since the last lo half
        # on its path (S' = S rounded up to a multiple of 256, the split strings);
        # 2 ops per multiply-add
        S = P // 8
        units = stages["schur_limb_macs"] / (nl * nl)   # entry x panel-column updates
        pairs = kara_digit_pairs(S, lv)
        ops = units * pairs * 2
        achieved = ops / (ms[6] * 1e-3) / 1e12
        kname = "k_upd_kara" if kara else "k_upd_mfma"
        out["roofline"] = {"bound": "mfma", "achieved": achieved, "peak": MFMA_INT8_PEAK_TOPS,
                           "unit": "TOP/s", "frac": achieved / MFMA_INT8_PEAK_TOPS,
                           "traffic": measured_traffic(workload, kname),
                           "kernel": kname + " (int8 ops of the algorithm, padding excluded)",
                           "launches": stages["launches"][1],
                           "avg_launch_ms": ms[6] / max(1, stages["launches"][1])}
    if a.form == "valu" and ms[0] > 0:
        achieved = stages["schur_limb_macs"] / (ms[0] * 1e-3)
        out["roofline"] = valu_roofline(ctx, achieved, "k_upd_valu (every Schur update of the step)")

    # adjoint on the same factorisation: d lambda_1 / d beta (after the timed steps)
    if not a.no_grad:
        from hankel_inputs import dmoments_dbeta
        dmu = dmoments_dbeta(beta, 2 * N - 1, P + 64)
        log("adjoint")
        ctx.set_timing(True)
        g = ctx.lambda_grad(fac, dmu)
        tg = ctx.timing()["ms"][8]
        ctx.set_timing(False)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        g = ctx.lambda_grad(fac, dmu)
        torch.cuda.synchronize()
        tg2 = (time.perf_counter() - t0) * 1e3
        out["adjoint"] = {"dlambda1_dbeta": g["dlambda1"], "ms": tg2, "device_ms": tg,
                          "time_to_dlambda1_dbeta_s": dt + tg2 * 1e-3}

    # the batched workload: 64 instances in one captured graph
    if not a.no_batch:
        from hankel_inputs import batch_configs
        from paper_1810_01478_amd.api import Batch
        cfg = batch_configs()
        log("batched workload", len(cfg))
        specs = [(moments(b, 2 * n - 1, p + 64), n, 8, p, 16, "mfma") for (b, n, p) in cfg]
        bt = Batch(ctx, specs)
        bt.launch()
        bt.results()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        bt.launch()
        rb = bt.results()
        tb = time.perf_counter() - t0
        bmacs = sum(schur_limb_macs(n, p // 32) for (b, n, p) in cfg)
        out["batch"] = {"workload": "64 instances, beta in {1/3,1/2,2/3,1}, N in [32,512], P = condition estimate "
                                    "+ 512 bits, k = 8 (seed 1810)",
                        "s": tb, "instances_per_s": len(cfg) / tb, "schur_limb_mac_per_s": bmacs / tb,
                        "all_ok": all(r["status"] == 0 for r in rb)}
        bt.close()
        del bt
        torch.cuda.empty_cache()

    # CPU oracle on a bounded sample, doubling as a parity check of its columns
    if not a.no_cpu:
        import hashlib
        cols = max(1, min(a.cpu_cols, N - 1))
        procs = cpu_workers()
        log("cpu oracle sample", cols, "pivots on", procs, "processes")
        fs, tcpu = cpu_sample(mu, N, k, P, E, cols, procs)
        ctx.sync(fac)
        nw_, NT = 2 * nl, fac.NT
        d = fac.d.view(-1)[:N * nw_].view(N, nw_).cpu().numpy()
        lv = fac.l.view(-1)
        ok = fac.h_list()[:cols] == fs.h and fac.s_list() == fs.s
        for i in range(cols):
            ok = ok and hashlib.sha256(d[i].tobytes()).hexdigest() == fs.d_sha[i]
            col = lv[(i * NT + i + 1) * nl:(i * NT + N) * nl].cpu().numpy()
            ok = ok and hashlib.sha256(col.tobytes()).hexdigest() == fs.b_sha[i]
        sample_macs = sample_limb_macs(N, cols, nl)
        out["cpu_baseline"] = {"value": sample_macs / tcpu, "unit": "limb-MAC/s", "cores": procs, "kind": "oracle",
                               "sample": "oracle (row-parallel contract, GMP multiply-subtract) on the first %d "
                                         "pivots of the same %dx%d matrix at P=%d: %.3g Schur limb-MACs in %.1f s "
                                         "of column loop on %d processes (matrix load excluded)"
                                         % (cols, N, N, P, sample_macs, tcpu, procs),
                               "parity_sample_columns_bit_exact": bool(ok)}
    # VALU sample: first two panels of the same matrix in both forms, bitwise
    if not a.no_valu and N > 32:
        cols = 32
        log("valu sample", cols, "columns")
        other = "valu" if a.form == "mfma" else "mfma"
        fac2 = ctx.alloc(ctx.shape(N, k, P, E, other))
        rates = {}
        for form, f in ((a.form, fac), (other, fac2)):
            ctx.set_timing(True)
            ctx.factor_cols(mu, N, k, P, E, form, 0, cols, fac=f, packed=packed)
            ctx.sync(f)
            t = ctx.timing()
            ctx.set_timing(False)
            rates[form] = t["schur_limb_macs"] / (t["ms"][0] * 1e-3)
        # the trailing matrix still to be factored: tiles (R, C) with C >= cols / 32
        # (the diagonal entries of factored columns are dead and the MFMA form's
        # pivot lookahead does not update them)
        so, tb = fac.sizes.trail_offset, 1024 * 2 * nl * 4
        same = bool(torch.equal(fac.l, fac2.l) and torch.equal(fac.d[:cols * 2 * nl], fac2.d[:cols * 2 * nl]))
        for R in range(cols // 32, fac.sizes.NT // 32):
            t0 = so + (R * (R + 1) // 2 + cols // 32) * tb
            t1 = so + (R * (R + 1) // 2 + R + 1) * tb
            same = same and bool(torch.equal(fac.ws[t0:t1], fac2.ws[t0:t1]))
        out["valu_sample"] = {"columns": cols, "mfma_limb_mac_per_s": rates["mfma"],
                              "valu_limb_mac_per_s": rates["valu"], "mfma_over_valu": rates["mfma"] / rates["valu"],
                              "bit_identical": same}
        if a.form == "mfma":
            out["roofline_valu"] = valu_roofline(ctx, rates["valu"], "k_upd_valu (Schur updates of the first %d "
                                                                     "pivots of the same matrix)" % cols)
        del fac2
        torch.cuda.empty_cache()

    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
