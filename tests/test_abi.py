"""The C ABI library loads and exports every entry point include/hl.h declares;
the host-only size and argument checks work without a GPU."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hl.h")


def declared():
    src = open(HEADER).read()
    return sorted(set(re.findall(r"\b(hl_[a-z_]+)\s*\(", src)) - {"hl_status"})


def test_header_declares_the_path():
    names = declared()
    for n in ("hl_factor", "hl_inv_block", "hl_lambda_min", "hl_create", "hl_get_sizes"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_1810_01478_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("libhankel.so not built")
    lib = ctypes.CDLL(_lib.LIB_PATH)
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing
    assert sorted(_lib.EXPORTS) == sorted(declared())


def test_sizes_and_argument_checks_on_host():
    from paper_1810_01478_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("libhankel.so not built")
    L = _lib.lib()
    out = _lib.hl_sizes()
    sh = _lib.hl_shape(N=1024, k=16, prec_bits=49152, exp_block=16, form=0)
    assert L.hl_get_sizes(ctypes.byref(sh), ctypes.byref(out)) == _lib.HL_OK
    assert out.nl == 1536 and out.NT == 1024
    assert out.l_words == 1024 * 1024 * 1536
    # trailing matrix: 528 tiles of 32 x 32 entries of 2 nl limbs
    assert out.trail_bytes == 528 * 1024 * 3072 * 4
    assert out.workspace_bytes > out.trail_bytes
    for bad in (dict(N=0), dict(k=0), dict(k=40), dict(prec_bits=1000), dict(prec_bits=128),
                dict(exp_block=0), dict(form=7), dict(N=8193)):
        kw = dict(N=64, k=8, prec_bits=2048, exp_block=16, form=1)
        kw.update(bad)
        s = _lib.hl_shape(**kw)
        assert L.hl_get_sizes(ctypes.byref(s), ctypes.byref(out)) == _lib.HL_EINVAL, bad
        assert L.hl_last_error()
    assert L.hl_factor(None, ctypes.byref(sh), None, None, 1, None, 0, None, None) == _lib.HL_EINVAL
    assert L.hl_set_karatsuba(None, 0) == _lib.HL_EINVAL
