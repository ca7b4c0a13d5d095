"""ctypes binding of libhankel.so (include/hl.h).  Argument marshalling only:
every step of the path runs in the library's HIP kernels.  Loading fails loudly
when the library is missing; there is no fallback."""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhankel.so")

HL_OK, HL_EINVAL, HL_ENOTPD, HL_EOVERFLOW, HL_ENOCONV, HL_EHIP, HL_ENOMEM = range(7)
HL_FORM_MFMA8, HL_FORM_VALU = 0, 1
STATUS_NAMES = {0: "HL_OK", 1: "HL_EINVAL", 2: "HL_ENOTPD", 3: "HL_EOVERFLOW", 4: "HL_ENOCONV",
                5: "HL_EHIP", 6: "HL_ENOMEM"}

EXPORTS = ["hl_create", "hl_destroy", "hl_last_error", "hl_get_sizes", "hl_factor", "hl_factor_cols", "hl_inv_block",
           "hl_lambda_min", "hl_lambda_min_noalloc", "hl_lambda_next", "hl_sync", "hl_set_timing", "hl_set_karatsuba", "hl_set_eig_maxit", "hl_get_timing", "hl_debug_mul", "hl_debug_recip", "hl_debug_valu_peak",
           "hl_debug_mfma_layout", "hl_debug_mul_wg", "hl_lambda_grad", "hl_batch_plan_bytes", "hl_batch_create", "hl_batch_launch",
           "hl_batch_results", "hl_batch_destroy", "hl_autotune"]


class hl_shape(ctypes.Structure):
    _fields_ = [("N", ctypes.c_int32), ("k", ctypes.c_int32), ("prec_bits", ctypes.c_int32),
                ("exp_block", ctypes.c_int32), ("form", ctypes.c_int32)]


class hl_sizes(ctypes.Structure):
    _fields_ = [("workspace_bytes", ctypes.c_size_t), ("d_words", ctypes.c_size_t),
                ("l_words", ctypes.c_size_t), ("x_words", ctypes.c_size_t),
                ("blk_words", ctypes.c_size_t), ("nl", ctypes.c_int32), ("NT", ctypes.c_int32),
                ("mu_limbs_min", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("trail_offset", ctypes.c_size_t), ("trail_bytes", ctypes.c_size_t),
                ("diag_offset", ctypes.c_size_t)]


class hl_factor_t(ctypes.Structure):
    _fields_ = [("d", ctypes.c_void_p), ("h", ctypes.c_void_p), ("s", ctypes.c_void_p),
                ("l", ctypes.c_void_p)]


class hl_lambda_t(ctypes.Structure):
    _fields_ = [("lambda1", ctypes.c_double), ("lambda1_km1", ctypes.c_double),
                ("trunc", ctypes.c_double), ("exp", ctypes.c_int64), ("exp_km1", ctypes.c_int64),
                ("iterations", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class hl_lambda_j_t(ctypes.Structure):
    _fields_ = [("lambda_", ctypes.c_double), ("lambda_km1", ctypes.c_double),
                ("trunc", ctypes.c_double), ("exp", ctypes.c_int64), ("exp_km1", ctypes.c_int64),
                ("j", ctypes.c_int32), ("iterations", ctypes.c_int32)]


class hl_timing_t(ctypes.Structure):
    _fields_ = [("ms", ctypes.c_double * 12), ("launches", ctypes.c_int64 * 4),
                ("schur_limb_macs", ctypes.c_double)]


class hl_grad_t(ctypes.Structure):
    _fields_ = [("dlambda1", ctypes.c_double), ("lambda1", ctypes.c_double), ("ynorm", ctypes.c_double),
                ("z_shift", ctypes.c_int64), ("num_shift", ctypes.c_int64), ("num_offset", ctypes.c_uint64),
                ("den_offset", ctypes.c_uint64), ("num_limbs", ctypes.c_int32), ("den_limbs", ctypes.c_int32)]


class hl_instance(ctypes.Structure):
    _fields_ = [("shape", hl_shape), ("mu", ctypes.c_void_p), ("mu_exp", ctypes.c_void_p), ("w", ctypes.c_int32),
                ("ws", ctypes.c_void_p), ("ws_bytes", ctypes.c_size_t), ("f", hl_factor_t), ("x", ctypes.c_void_p),
                ("blk", ctypes.c_void_p), ("blk_exp", ctypes.c_void_p)]


class hl_tune_t(ctypes.Structure):
    _fields_ = [("items_per_simd", ctypes.c_int32), ("range_cap", ctypes.c_int32),
                ("valu_below_bits", ctypes.c_int32), ("karatsuba", ctypes.c_int32)]


class HLError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s: %s" % (STATUS_NAMES.get(code, code), msg))
        self.code = code


_lib = None


def lib():
    """The loaded library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libhankel.so is not built (run paper_1810_01478_amd.build)")
        L = ctypes.CDLL(LIB_PATH)
        P, I32, I64, SZ = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
        sig = {
            "hl_create": [ctypes.POINTER(ctypes.c_void_p), ctypes.c_int],
            "hl_destroy": [P],
            "hl_get_sizes": [ctypes.POINTER(hl_shape), ctypes.POINTER(hl_sizes)],
            "hl_factor": [P, ctypes.POINTER(hl_shape), P, P, I32, P, SZ, ctypes.POINTER(hl_factor_t), P],
            "hl_factor_cols": [P, ctypes.POINTER(hl_shape), P, P, I32, P, SZ, ctypes.POINTER(hl_factor_t),
                               I32, I32, P],
            "hl_inv_block": [P, ctypes.POINTER(hl_shape), ctypes.POINTER(hl_factor_t), P, SZ, P, P, P, P],
            "hl_lambda_min": [P, ctypes.POINTER(hl_shape), P, P, P, SZ, P, P, ctypes.POINTER(hl_lambda_t), P],
            "hl_lambda_min_noalloc": [P, ctypes.POINTER(hl_shape), P, P, P, P, ctypes.POINTER(hl_lambda_t), P],
            "hl_lambda_next": [P, ctypes.POINTER(hl_shape), P, P, P, SZ, ctypes.c_int32, P, P,
                               ctypes.POINTER(hl_lambda_j_t), P],
            "hl_sync": [P, P, P, ctypes.POINTER(I32)],
            "hl_set_timing": [P, ctypes.c_int],
            "hl_set_karatsuba": [P, ctypes.c_int32],
            "hl_set_eig_maxit": [P, ctypes.c_int32],
            "hl_get_timing": [P, ctypes.POINTER(hl_timing_t)],
            "hl_debug_mul": [P, I32, P, I32, P, I32, P],
            "hl_debug_recip": [P, I32, I32, P, P, P],
            "hl_debug_valu_peak": [I32, I32, I32, P, P],
            "hl_debug_mfma_layout": [P, P],
            "hl_debug_mul_wg": [P, I32, P, I32, P, I32, I32, P],
            "hl_lambda_grad": [P, ctypes.POINTER(hl_shape), ctypes.POINTER(hl_factor_t), P, P, P, P, P, I32, P, SZ,
                               P, ctypes.POINTER(hl_grad_t), P],
            "hl_batch_plan_bytes": [I32, ctypes.POINTER(hl_instance), ctypes.POINTER(hl_tune_t),
                                    ctypes.POINTER(ctypes.c_size_t)],
            "hl_batch_create": [P, I32, ctypes.POINTER(hl_instance), ctypes.POINTER(hl_tune_t), P, SZ,
                                ctypes.POINTER(ctypes.c_void_p)],
            "hl_batch_launch": [P, P],
            "hl_batch_results": [P, P, ctypes.POINTER(hl_lambda_t), ctypes.POINTER(ctypes.c_int)],
            "hl_batch_destroy": [P],
            "hl_autotune": [P, I32, ctypes.POINTER(hl_instance), P, SZ, I32, ctypes.POINTER(hl_tune_t),
                            ctypes.POINTER(ctypes.c_double)],
        }
        for name, args in sig.items():
            try:
                f = getattr(L, name)
            except AttributeError:
                continue
            f.argtypes = args
            f.restype = ctypes.c_int
        L.hl_last_error.restype = ctypes.c_char_p
        L.hl_last_error.argtypes = []
        _lib = L
    return _lib


def check(code):
    if code != HL_OK:
        raise HLError(code, lib().hl_last_error().decode())
    return code
