"""Python front end of libhankel: torch supplies device memory and the stream,
the library does all the arithmetic.

    ctx = Context()
    fac = ctx.factor(moments(Fraction(1, 2), 127), N=64, k=8, P=2048)
    res = ctx.lambda_min(fac)          # factor -> block -> eigen-step
"""
from __future__ import annotations

import ctypes
import math
from dataclasses import dataclass, field
from fractions import Fraction
from typing import List, Optional, Sequence

import numpy as np
import torch

from hankel_inputs import moments as _moments, pack_limbs, unpack_limbs

from . import _lib as L

FORMS = {"mfma": L.HL_FORM_MFMA8, "mfma8": L.HL_FORM_MFMA8, "valu": L.HL_FORM_VALU}


def _ptr(t: torch.Tensor) -> ctypes.c_void_p:
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream=None) -> ctypes.c_void_p:
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _u32_tensor(arr: np.ndarray, device) -> torch.Tensor:
    return torch.from_numpy(np.ascontiguousarray(arr, dtype=np.uint32).view(np.int32)).to(device)


def _ints(t: torch.Tensor, limbs: int, signed: bool) -> List[int]:
    a = t.detach().cpu().numpy().view(np.uint32).reshape(-1, limbs)
    return unpack_limbs(a, signed=signed)


@dataclass
class Factorization:
    shape: L.hl_shape
    sizes: L.hl_sizes
    ws: torch.Tensor
    d: torch.Tensor
    h: torch.Tensor
    s: torch.Tensor
    l: torch.Tensor
    x: Optional[torch.Tensor] = None
    blk: Optional[torch.Tensor] = None
    blk_exp: Optional[torch.Tensor] = None
    views: L.hl_factor_t = field(default_factory=L.hl_factor_t)

    @property
    def N(self):
        return self.shape.N

    @property
    def nl(self):
        return self.sizes.nl

    @property
    def NT(self):
        return self.sizes.NT

    # host views for checks ---------------------------------------------------
    def pivots(self) -> List[int]:
        return _ints(self.d, 2 * self.nl, signed=True)

    def h_list(self) -> List[int]:
        return self.h.cpu().tolist()

    def s_list(self) -> List[int]:
        return self.s.cpu().tolist()

    def multipliers(self, i: int, rows: Optional[Sequence[int]] = None) -> List[int]:
        """b_ri for the given rows (default: all rows r > i) of column i."""
        nl, NT = self.nl, self.NT
        col = self.l.view(-1)[i * NT * nl:(i + 1) * NT * nl]
        vals = _ints(col, nl, signed=True)
        if rows is None:
            rows = range(i + 1, self.N)
        return [vals[r] for r in rows]

    def block(self):
        k, nl = self.shape.k, self.nl
        vals = _ints(self.blk, nl, signed=True)
        return [vals[a * k:(a + 1) * k] for a in range(k)], int(self.blk_exp.cpu().item())

    def linv(self):
        k, nl = self.shape.k, self.nl
        vals = _ints(self.x, nl, signed=True)
        return [vals[r * k:(r + 1) * k] for r in range(self.N)]


class Context:
    """One device, one library context."""

    def __init__(self, device: int = 0):
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU visible: libhankel runs on gfx950 only")
        self.device = torch.device("cuda", device)
        h = ctypes.c_void_p()
        L.check(L.lib().hl_create(ctypes.byref(h), device))
        self.h = h

    def close(self):
        if self.h:
            L.lib().hl_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------------------
    @staticmethod
    def shape(N, k, P, E=16, form="mfma") -> L.hl_shape:
        return L.hl_shape(N=N, k=k, prec_bits=P, exp_block=E, form=FORMS[form] if isinstance(form, str) else form)

    @staticmethod
    def sizes(sh: L.hl_shape) -> L.hl_sizes:
        out = L.hl_sizes()
        L.check(L.lib().hl_get_sizes(ctypes.byref(sh), ctypes.byref(out)))
        return out

    def pack_moments(self, mu):
        mants = [m.M for m in mu]
        if any(v <= 0 for v in mants):
            raise ValueError("moments must be positive")
        w = max(1, max((v.bit_length() + 31) // 32 for v in mants))
        limbs = _u32_tensor(pack_limbs(mants, w), self.device)
        exps = torch.tensor([m.e for m in mu], dtype=torch.int64, device=self.device)
        return limbs, exps, w

    def alloc(self, sh: L.hl_shape) -> Factorization:
        sz = self.sizes(sh)
        dev = self.device
        ws = torch.empty(sz.workspace_bytes, dtype=torch.uint8, device=dev)
        d = torch.empty(sz.d_words, dtype=torch.int32, device=dev)
        h = torch.empty(sh.N, dtype=torch.int32, device=dev)
        s = torch.empty(sh.N, dtype=torch.int32, device=dev)
        l = torch.empty(sz.l_words, dtype=torch.int32, device=dev)
        f = Factorization(shape=sh, sizes=sz, ws=ws, d=d, h=h, s=s, l=l)
        f.views = L.hl_factor_t(d=d.data_ptr(), h=h.data_ptr(), s=s.data_ptr(), l=l.data_ptr())
        f.x = torch.empty(max(1, sz.x_words), dtype=torch.int32, device=dev)
        f.blk = torch.empty(max(1, sz.blk_words), dtype=torch.int32, device=dev)
        f.blk_exp = torch.zeros(1, dtype=torch.int64, device=dev)
        return f

    def factor(self, mu, N, k, P, E=16, form="mfma", fac: Optional[Factorization] = None,
               packed=None, stream=None) -> Factorization:
        sh = self.shape(N, k, P, E, form)
        if fac is None:
            fac = self.alloc(sh)
        fac.shape = sh
        limbs, exps, w = packed if packed is not None else self.pack_moments(mu[:2 * N - 1])
        fac._mu = (limbs, exps, w)
        L.check(L.lib().hl_factor(self.h, ctypes.byref(sh), _ptr(limbs), _ptr(exps), w, _ptr(fac.ws),
                                  fac.ws.numel(), ctypes.byref(fac.views), _stream(stream)))
        return fac

    def factor_cols(self, mu, N, k, P, E, form, col_begin, col_end, fac: Optional[Factorization] = None,
                    packed=None, stream=None) -> Factorization:
        sh = self.shape(N, k, P, E, form)
        if fac is None:
            fac = self.alloc(sh)
        fac.shape = sh
        limbs, exps, w = packed if packed is not None else self.pack_moments(mu[:2 * N - 1])
        fac._mu = (limbs, exps, w)
        L.check(L.lib().hl_factor_cols(self.h, ctypes.byref(sh), _ptr(limbs), _ptr(exps), w, _ptr(fac.ws),
                                       fac.ws.numel(), ctypes.byref(fac.views), col_begin, col_end,
                                       _stream(stream)))
        return fac

    def sync(self, fac: Factorization, stream=None):
        idx = ctypes.c_int32(0)
        code = L.lib().hl_sync(self.h, _ptr(fac.ws), _stream(stream), ctypes.byref(idx))
        if code != L.HL_OK:
            raise L.HLError(code, L.lib().hl_last_error().decode() + " (index %d)" % idx.value)

    def inv_block(self, fac: Factorization, stream=None) -> Factorization:
        L.check(L.lib().hl_inv_block(self.h, ctypes.byref(fac.shape), ctypes.byref(fac.views), _ptr(fac.ws),
                                     fac.ws.numel(), _ptr(fac.x), _ptr(fac.blk), _ptr(fac.blk_exp),
                                     _stream(stream)))
        return fac

    def eigen(self, fac: Factorization, want_mant=True, stream=None):
        out = L.hl_lambda_t()
        nl = fac.nl
        m1 = torch.zeros(nl, dtype=torch.int32, device=self.device) if want_mant else None
        m2 = torch.zeros(nl, dtype=torch.int32, device=self.device) if want_mant else None
        code = L.lib().hl_lambda_min(self.h, ctypes.byref(fac.shape), _ptr(fac.blk), _ptr(fac.blk_exp),
                                     _ptr(fac.ws), fac.ws.numel(),
                                     _ptr(m1) if m1 is not None else None,
                                     _ptr(m2) if m2 is not None else None,
                                     ctypes.byref(out), _stream(stream))
        if code != L.HL_OK:
            raise L.HLError(code, L.lib().hl_last_error().decode())
        res = {"lambda1": out.lambda1, "lambda1_km1": out.lambda1_km1, "trunc": out.trunc,
               "exp": out.exp, "exp_km1": out.exp_km1, "iterations": out.iterations}
        off = fac.sizes.diag_offset
        fl = fac.ws[off:off + 256].view(torch.int32).cpu().tolist()
        res["trace"] = [fl[16:40], fl[40:64]]
        if want_mant:
            res["mant"] = _ints(m1, nl, signed=False)[0]
            res["mant_km1"] = _ints(m2, nl, signed=False)[0]
        return res

    def eigen_noalloc(self, fac: Factorization, want_mant=True, stream=None):
        """The eigen-step of eigen() through hl_lambda_min_noalloc: the same
        results from the block alone, its scratch in the library's static
        device array instead of the workspace."""
        out = L.hl_lambda_t()
        nl = fac.nl
        m1 = torch.zeros(nl, dtype=torch.int32, device=self.device) if want_mant else None
        m2 = torch.zeros(nl, dtype=torch.int32, device=self.device) if want_mant else None
        L.check(L.lib().hl_lambda_min_noalloc(self.h, ctypes.byref(fac.shape), _ptr(fac.blk), _ptr(fac.blk_exp),
                                              _ptr(m1) if m1 is not None else None,
                                              _ptr(m2) if m2 is not None else None,
                                              ctypes.byref(out), _stream(stream)))
        res = {"lambda1": out.lambda1, "lambda1_km1": out.lambda1_km1, "trunc": out.trunc,
               "exp": out.exp, "exp_km1": out.exp_km1, "iterations": out.iterations}
        if want_mant:
            res["mant"] = _ints(m1, nl, signed=False)[0]
            res["mant_km1"] = _ints(m2, nl, signed=False)[0]
        return res

    def lambda_min(self, fac: Factorization, stream=None):
        self.inv_block(fac, stream)
        return self.eigen(fac, stream=stream)

    def lambda_next(self, fac: Factorization, count: int = 2, want_mant=True, stream=None):
        """lambda_2 (and lambda_3) with their truncation estimates (hl_lambda_next);
        needs lambda_min(fac) first.  One dict per eigenvalue, j = 2, 3."""
        nl = fac.nl
        out = (L.hl_lambda_j_t * count)()
        m1 = torch.zeros(count * nl, dtype=torch.int32, device=self.device) if want_mant else None
        m2 = torch.zeros(count * nl, dtype=torch.int32, device=self.device) if want_mant else None
        L.check(L.lib().hl_lambda_next(self.h, ctypes.byref(fac.shape), _ptr(fac.blk), _ptr(fac.blk_exp),
                                       _ptr(fac.ws), fac.ws.numel(), count,
                                       _ptr(m1) if m1 is not None else None,
                                       _ptr(m2) if m2 is not None else None, out, _stream(stream)))
        res = []
        for i in range(count):
            o = out[i]
            r = {"j": o.j, "lambda": o.lambda_, "lambda_km1": o.lambda_km1, "trunc": o.trunc, "exp": o.exp,
                 "exp_km1": o.exp_km1, "iterations": o.iterations}
            if want_mant:
                r["mant"] = _ints(m1[i * nl:(i + 1) * nl], nl, signed=False)[0]
                r["mant_km1"] = _ints(m2[i * nl:(i + 1) * nl], nl, signed=False)[0]
            res.append(r)
        return res

    def pack_signed(self, vals):
        """Signed dyadics (M, e) as magnitude limbs, exponents and sign flags."""
        mags = [abs(v.M) for v in vals]
        w = max(1, max((m.bit_length() + 31) // 32 for m in mags))
        limbs = _u32_tensor(pack_limbs(mags, w), self.device)
        exps = torch.tensor([v.e for v in vals], dtype=torch.int64, device=self.device)
        neg = torch.tensor([1 if v.M < 0 else 0 for v in vals], dtype=torch.int32, device=self.device)
        return limbs, exps, neg, w

    def lambda_grad(self, fac: Factorization, dmu, want_z: bool = False, stream=None):
        """sum_m (d lambda_1 / d mu_m) dmu_m on the GPU (hl_lambda_grad); with
        dmu = d mu / d beta this is d lambda_1 / d beta.  Needs lambda_min(fac)
        first."""
        N, nl = fac.N, fac.nl
        limbs, exps, neg, w = self.pack_signed(dmu[:2 * N - 1])
        z = torch.zeros(N * nl, dtype=torch.int32, device=self.device) if want_z else None
        out = L.hl_grad_t()
        L.check(L.lib().hl_lambda_grad(self.h, ctypes.byref(fac.shape), ctypes.byref(fac.views), _ptr(fac.x),
                                       _ptr(fac.blk_exp), _ptr(limbs), _ptr(exps), _ptr(neg), w, _ptr(fac.ws),
                                       fac.ws.numel(), _ptr(z) if z is not None else None, ctypes.byref(out),
                                       _stream(stream)))
        res = {"dlambda1": out.dlambda1, "lambda1": out.lambda1, "ynorm": out.ynorm, "z_shift": out.z_shift,
               "num_shift": out.num_shift}
        if out.num_limbs:
            a, b = out.num_offset, out.den_offset
            res["num"] = _ints(fac.ws[a:a + 4 * out.num_limbs].view(torch.int32), out.num_limbs, signed=True)[0]
            res["den"] = _ints(fac.ws[b:b + 4 * out.den_limbs].view(torch.int32), out.den_limbs, signed=False)[0]
        if want_z:
            res["z"] = _ints(z, nl, signed=True)
        return res

    # timing ------------------------------------------------------------------
    def set_timing(self, on: bool):
        L.check(L.lib().hl_set_timing(self.h, 1 if on else 0))

    def set_karatsuba(self, mode: int):
        """Schur-update form of later factorisations of MFMA shapes: 0 digit
        product, 1 or 2 Karatsuba levels (P % 256 == 0, P % 512 == 0), -1 by
        precision (the default)."""
        L.check(L.lib().hl_set_karatsuba(self.h, int(mode)))

    def set_eig_maxit(self, maxit: int):
        """Iteration limit of the eigen-step per block (0: the default); a
        smaller one makes eigen() raise HL_ENOCONV (exercises that path)."""
        L.check(L.lib().hl_set_eig_maxit(self.h, int(maxit)))

    def timing(self):
        t = L.hl_timing_t()
        L.check(L.lib().hl_get_timing(self.h, ctypes.byref(t)))
        return {"ms": list(t.ms), "launches": list(t.launches), "schur_limb_macs": t.schur_limb_macs}

    # test hooks ----------------------------------------------------------------
    def debug_mul(self, a: int, b: int, na: int, nb: int, nout: int) -> int:
        A = _u32_tensor(pack_limbs([a], na), self.device)
        B = _u32_tensor(pack_limbs([b], nb), self.device)
        O = torch.zeros(nout, dtype=torch.int32, device=self.device)
        L.check(L.lib().hl_debug_mul(_ptr(A), na, _ptr(B), nb, _ptr(O), nout, _stream()))
        torch.cuda.synchronize()
        return _ints(O, nout, signed=False)[0]

    def debug_mul_wg(self, a: int, b: int, na: int, nb: int, nout: int, threads: int = 1024) -> int:
        A = _u32_tensor(pack_limbs([a], na), self.device)
        B = _u32_tensor(pack_limbs([b], nb), self.device)
        O = torch.zeros(nout, dtype=torch.int32, device=self.device)
        L.check(L.lib().hl_debug_mul_wg(_ptr(A), na, _ptr(B), nb, _ptr(O), nout, threads, _stream()))
        torch.cuda.synchronize()
        return _ints(O, nout, signed=False)[0]

    def debug_mfma_layout(self):
        O = torch.zeros(2048, dtype=torch.int32, device=self.device)
        L.check(L.lib().hl_debug_mfma_layout(_ptr(O), _stream()))
        torch.cuda.synchronize()
        return O.cpu().tolist()

    def debug_valu_peak(self, mode: int = 1, blocks: int = 8192, iters: int = 8192, repeats: int = 3):
        """Rate of the VALU integer multiply-add (hl_debug_valu_peak): best of
        `repeats` launches, timed with events on the current stream.  Returns
        (multiply-adds per second, ms per launch)."""
        sink = torch.zeros(1, dtype=torch.int64, device=self.device)
        st = torch.cuda.current_stream()
        L.check(L.lib().hl_debug_valu_peak(mode, blocks, iters, _ptr(sink), _stream()))   # warm-up
        best = None
        for _ in range(repeats):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(st)
            L.check(L.lib().hl_debug_valu_peak(mode, blocks, iters, _ptr(sink), _stream()))
            e1.record(st)
            e1.synchronize()
            ms = e0.elapsed_time(e1)
            best = ms if best is None else min(best, ms)
        macs = blocks * 256.0 * iters * 8
        return macs / (best * 1e-3), best

    def debug_recip(self, d: int, P: int):
        nl = P // 32
        nd = max(1, (d.bit_length() + 31) // 32)
        D = _u32_tensor(pack_limbs([d], nd), self.device)
        O = torch.zeros(nl + 4, dtype=torch.int32, device=self.device)
        H = torch.zeros(1, dtype=torch.int32, device=self.device)
        L.check(L.lib().hl_debug_recip(_ptr(D), nd, P, _ptr(O), _ptr(H), _stream()))
        torch.cuda.synchronize()
        return _ints(O, nl + 4, signed=False)[0], int(H.cpu().item())


class Batch:
    """Many instances in one captured launch sequence (hl_batch_*).

    specs: list of (mu, N, k, P, E, form) with mu the moment dyadics.  The
    device buffers of every instance and the plan are held here; launch() replays
    the graph, results() waits and returns one dict per instance."""

    def __init__(self, ctx: "Context", specs, tune: Optional[dict] = None):
        self.ctx = ctx
        self.facs, self.packed = [], []
        n = len(specs)
        self.inst = (L.hl_instance * n)()
        for j, (mu, N, k, P, E, form) in enumerate(specs):
            sh = ctx.shape(N, k, P, E, form)
            fac = ctx.alloc(sh)
            limbs, exps, w = ctx.pack_moments(mu[:2 * N - 1])
            fac._mu = (limbs, exps, w)
            self.facs.append(fac)
            self.inst[j] = L.hl_instance(shape=sh, mu=limbs.data_ptr(), mu_exp=exps.data_ptr(), w=w,
                                         ws=fac.ws.data_ptr(), ws_bytes=fac.ws.numel(), f=fac.views,
                                         x=fac.x.data_ptr(), blk=fac.blk.data_ptr(), blk_exp=fac.blk_exp.data_ptr())
        self.tune = L.hl_tune_t(**tune) if tune else None
        nb = ctypes.c_size_t(0)
        tp = ctypes.byref(self.tune) if self.tune is not None else None
        L.check(L.lib().hl_batch_plan_bytes(n, self.inst, tp, ctypes.byref(nb)))
        self.plan = torch.empty(max(256, nb.value), dtype=torch.uint8, device=ctx.device)
        h = ctypes.c_void_p()
        L.check(L.lib().hl_batch_create(ctx.h, n, self.inst, tp, _ptr(self.plan), self.plan.numel(),
                                        ctypes.byref(h)))
        self.h = h

    def launch(self, stream=None):
        L.check(L.lib().hl_batch_launch(self.h, _stream(stream)))

    def results(self, stream=None):
        n = len(self.facs)
        out = (L.hl_lambda_t * n)()
        st = (ctypes.c_int * n)()
        code = L.lib().hl_batch_results(self.h, _stream(stream), out, st)
        res = []
        for j in range(n):
            o = out[j]
            res.append({"status": st[j], "lambda1": o.lambda1, "lambda1_km1": o.lambda1_km1, "trunc": o.trunc,
                        "exp": o.exp, "iterations": o.iterations})
        if code != L.HL_OK:
            raise L.HLError(code, L.lib().hl_last_error().decode())
        return res

    def close(self):
        if getattr(self, "h", None):
            L.lib().hl_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def autotune(batch: Batch, panels: int = 2):
    """Time candidate launch shapes on the batch's first panel steps (hl_autotune);
    returns (tuning dict, ms per replay).  The instances' workspaces serve as
    scratch (a later launch of the batch recomputes everything from the load);
    the plans go to a scratch buffer, not the batch's own."""
    best = L.hl_tune_t()
    ms = ctypes.c_double(0)
    scratch = torch.empty(2 * batch.plan.numel(), dtype=torch.uint8, device=batch.ctx.device)
    L.check(L.lib().hl_autotune(batch.ctx.h, len(batch.facs), batch.inst, _ptr(scratch), scratch.numel(),
                                panels, ctypes.byref(best), ctypes.byref(ms)))
    torch.cuda.synchronize()
    del scratch
    return ({"items_per_simd": best.items_per_simd, "range_cap": best.range_cap,
             "valu_below_bits": best.valu_below_bits, "karatsuba": best.karatsuba}, ms.value)


def lambda_min(beta, N: int, k: int, P: int, E: int = 16, form: str = "mfma", mant_bits: int = 0,
               ctx: Optional[Context] = None):
    """lambda_1 of H_N for the weight exp(-x^beta), end to end on the GPU."""
    ctx = ctx or Context()
    mu = _moments(beta, 2 * N - 1, mant_bits=mant_bits or 2 * P)
    fac = ctx.factor(mu, N, k, P, E, form)
    return ctx.lambda_min(fac)


class LambdaMin(torch.autograd.Function):
    """lambda_1(beta) of H_N for the weight exp(-x^beta) as a differentiable
    function of beta.  Forward: moments on the host, then factor -> block ->
    eigen-step on the GPU.  Backward: d mu / d beta on the host (digamma chain),
    then the adjoint kernels (hl_lambda_grad) give d lambda_1 / d beta.

    beta is a 0-dim float64 tensor; its value is read as the shortest decimal
    that prints as it (0.45 -> 9/20), exactly, so the moments are those of that
    rational.  A value whose decimal has a reduced denominator above 10**6 (for
    example 0.1234567891) raises ValueError instead of being snapped to a nearby
    rational, so lambda_1 and its derivative are never those of another beta."""

    @staticmethod
    def forward(ctx_, beta, N, k, P, E, form, context):
        from hankel_inputs.moments import _as_fraction
        b = _as_fraction(float(beta.detach().cpu().item()))
        mu = _moments(b, 2 * N - 1, mant_bits=P + 64)
        fac = context.factor(mu, N, k, P, E, form)
        res = context.lambda_min(fac)
        ctx_.state = (context, fac, b, N, P)
        return torch.tensor(res["lambda1"], dtype=torch.float64, device=beta.device)

    @staticmethod
    def backward(ctx_, grad):
        from hankel_inputs import dmoments_dbeta
        context, fac, b, N, P = ctx_.state
        dmu = dmoments_dbeta(b, 2 * N - 1, P + 64)
        g = context.lambda_grad(fac, dmu)["dlambda1"]
        return grad * g, None, None, None, None, None, None


def lambda1(beta: torch.Tensor, N: int, k: int, P: int, E: int = 16, form: str = "mfma",
            context: Optional[Context] = None) -> torch.Tensor:
    """Differentiable lambda_1(beta) (see LambdaMin)."""
    return LambdaMin.apply(beta, N, k, P, E, form, context or Context())
