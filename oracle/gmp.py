"""Multiply-subtract on GMP integers through ctypes, for the oracle at large sizes.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

The contract's Schur update (Algorithm 1, inner loops) is a long run of exact
operations a <- a - b u on integers of thousands of bits.  Python integers do
this correctly but slowly; GMP's mpz_submul does the same exact operation about
ten times faster.  This module is nothing but that library primitive: an mpz
that can be filled from and read back into a Python int, and the exact
operations a -= b u, a += b u.  No rounding, scaling or step of the method lives
here; the contract (``oracle/contract.py``) and the row-parallel runner
(``oracle/parallel.py``) decide what is computed.

GMP's C header is not installed here, so the few entry points used are declared
by hand: ``mpz_t`` is {int alloc; int size; limb pointer}, with |size| the
number of 64-bit limbs in use and its sign the sign of the number.

Parity status: pinned in ``tests/test_oracle_gmp.py`` against Python's own
integer arithmetic (an independent implementation) on random operands of both
signs, zero, and sizes from one limb to 200,000 bits.
"""

from __future__ import annotations

import ctypes
import ctypes.util

_F = None   # the GMP entry points by short name


class _mpz(ctypes.Structure):
    _fields_ = [("alloc", ctypes.c_int), ("size", ctypes.c_int), ("d", ctypes.c_void_p)]


def lib():
    """The entry points, looked up by their exported names (__gmpz_*)."""
    global _F
    if _F is None:
        name = ctypes.util.find_library("gmp") or "libgmp.so.10"
        g = ctypes.CDLL(name)
        P = ctypes.POINTER(_mpz)
        sig = {
            "init": ([P], None), "clear": ([P], None), "submul": ([P, P, P], None),
            "addmul": ([P, P, P], None), "neg": ([P, P], None),
            "import": ([P, ctypes.c_size_t, ctypes.c_int, ctypes.c_size_t, ctypes.c_int, ctypes.c_size_t,
                        ctypes.c_void_p], None),
            "export": ([ctypes.c_void_p, ctypes.POINTER(ctypes.c_size_t), ctypes.c_int, ctypes.c_size_t,
                        ctypes.c_int, ctypes.c_size_t, P], ctypes.c_void_p),
        }
        F = {}
        for short, (args, res) in sig.items():
            fn = getattr(g, "__gmpz_" + short)
            fn.argtypes = args
            fn.restype = res
            F[short] = fn
        _F = F
    return _F


def available() -> bool:
    try:
        lib()
        return True
    except (OSError, AttributeError):
        return False


class Mpz:
    """One GMP integer.  ``set`` and ``get`` convert from and to Python ints
    (magnitude as little-endian bytes, sign kept apart)."""

    __slots__ = ("z", "ref")

    def __init__(self, value: int = 0):
        self.z = _mpz()
        self.ref = ctypes.byref(self.z)
        lib()["init"](self.ref)
        if value:
            self.set(value)

    def __del__(self):
        if _F is not None and self.ref is not None:
            _F["clear"](self.ref)
            self.ref = None

    def set(self, value: int) -> None:
        F = lib()
        mag = -value if value < 0 else value
        raw = mag.to_bytes(max(1, (mag.bit_length() + 7) // 8), "little")
        F["import"](self.ref, len(raw), -1, 1, 0, 0, raw)
        if value < 0:
            F["neg"](self.ref, self.ref)

    def set_bytes(self, addr: int, nbytes: int, negative: bool) -> None:
        """From a little-endian magnitude of nbytes bytes at a raw address."""
        F = lib()
        F["import"](self.ref, nbytes, -1, 1, 0, 0, ctypes.c_void_p(addr))
        if negative:
            F["neg"](self.ref, self.ref)

    def get(self) -> int:
        size = self.z.size
        if size == 0:
            return 0
        nbytes = 8 * abs(size)
        buf = (ctypes.c_ubyte * nbytes)()
        count = ctypes.c_size_t(0)
        lib()["export"](buf, ctypes.byref(count), -1, 1, 0, 0, self.ref)
        mag = int.from_bytes(bytes(buf)[:count.value], "little")
        return -mag if size < 0 else mag

    def submul(self, b: "Mpz", u: "Mpz") -> None:
        """self -= b u, exactly."""
        _F["submul"](self.ref, b.ref, u.ref)

    def addmul(self, b: "Mpz", u: "Mpz") -> None:
        """self += b u, exactly."""
        _F["addmul"](self.ref, b.ref, u.ref)


def submul_int(a: int, b: int, u: int) -> int:
    """a - b u for Python ints through GMP (the contract's ``submul`` hook)."""
    x = Mpz(a)
    x.submul(Mpz(b), Mpz(u))
    return x.get()
