"""MI355X-native extreme-precision Hankel LDL^T -> k x k block of H^-1 -> lambda_1.

The arithmetic lives in libhankel.so (HIP kernels for gfx950, C ABI in
include/hl.h); this package is its Python front end.  Import of the front end is
lazy so that the build step and CPU-only tooling do not need a GPU.
"""
__all__ = ["Context", "lambda_min", "lambda1", "LambdaMin", "build"]


def __getattr__(name):
    if name in ("Context", "lambda_min", "lambda1", "LambdaMin", "Factorization"):
        from . import api
        return getattr(api, name)
    raise AttributeError(name)
