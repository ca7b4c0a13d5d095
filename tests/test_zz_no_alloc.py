"""hl_lambda_min_noalloc (the eigen-step with its scratch in the library's
static device array) against hl_lambda_min (scratch in the caller's
workspace): the same kernels, so the same bits.  Two calls in a row, the second
on a smaller shape, so the second runs on what the first left in the array."""
import ctypes
from fractions import Fraction

import pytest

from hankel_inputs import moments

from gpu_util import ctx, say

pytestmark = pytest.mark.gpu

CASES = [  # beta, N, k, P, E, form: the second smaller in every size
    (Fraction(1, 2), 96, 12, 4096, 16, "mfma"),
    (Fraction(1, 3), 40, 6, 1024, 1, "valu"),
]

KEYS = ("lambda1", "lambda1_km1", "trunc", "exp", "exp_km1", "iterations", "mant", "mant_km1")


def test_noalloc_equals_workspace_eigen_step_twice():
    c = ctx()
    for beta, N, k, P, E, form in CASES:
        say("noalloc eigen-step", beta, N, k, P, E, form)
        mu = moments(beta, 2 * N - 1)
        fac = c.factor(mu, N, k, P, E, form)
        ref = c.lambda_min(fac)
        got = c.eigen_noalloc(fac)
        for key in KEYS:
            assert got[key] == ref[key], (key, got[key], ref[key])
        assert ref["lambda1"] > 0 and ref["trunc"] <= 0


def test_noalloc_refuses_shapes_beyond_its_scratch():
    from paper_1810_01478_amd import _lib as L
    c = ctx()
    sh = L.hl_shape(N=64, k=32, prec_bits=32768, exp_block=16, form=0)
    out = L.hl_lambda_t()
    code = L.lib().hl_lambda_min_noalloc(c.h, ctypes.byref(sh), ctypes.c_void_p(16), ctypes.c_void_p(16),
                                         None, None, ctypes.byref(out), None)
    assert code == L.HL_EINVAL
    assert b"scratch" in L.lib().hl_last_error()
