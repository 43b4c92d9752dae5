"""ctypes view of the C ABI in include/ttcconv.h (libttcconv.so).

Only marshalling lives here: struct layouts, symbol signatures and loading.
Loading fails loudly when the library has not been built; there is no
fallback implementation.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

# the in-tree build; TC_LIBRARY names another build of the same library (the
# host-sanitizer build of `build.build_sanitized`, for instance)
LIB_PATH = os.environ.get("TC_LIBRARY") or os.path.join(os.path.dirname(os.path.abspath(__file__)), "libttcconv.so")

TC_OK, TC_SINGULAR, TC_NEED_PREV, TC_NONFINITE = 0, 1, 2, 3
TC_EINVAL, TC_ESHAPE, TC_EDTYPE, TC_EOVERFLOW, TC_ENOMEM, TC_EDEVICE = -1, -2, -3, -4, -5, -6
TC_U8, TC_F16, TC_F32, TC_I32, TC_F64 = 0, 1, 2, 3, 4
TC_FULL, TC_SAME, TC_VALID = 0, 1, 2
TC_MAX_DIMS = 8
TC_MAX_LEVELS = 4
TC_NUM_SUMS = 10

MODES = {"full": TC_FULL, "same": TC_SAME, "valid": TC_VALID}
TC_PHASE_FUSED, TC_PHASE_FINISH = 1, 2
TC_STENCIL_FD2, TC_STENCIL_ROBERTS, TC_STENCIL_PREWITT3, TC_STENCIL_SOBEL3 = 0, 1, 2, 3
TC_SELECT_DECREASING_TTC, TC_SELECT_MIN_RESIDUAL = 0, 1
TC_LOWPASS_NONE, TC_LOWPASS_BINOMIAL3 = 0, 1
TC_CONV_AUTO, TC_CONV_DIRECT, TC_CONV_FFT = 0, 1, 2
TC_NOALLOC_SCRATCH_BYTES = 4 << 20
METHODS = {"auto": TC_CONV_AUTO, "direct": TC_CONV_DIRECT, "fft": TC_CONV_FFT}


class TcTensor(C.Structure):
    _fields_ = [
        ("data", C.c_void_p),
        ("dtype", C.c_int32),
        ("ndim", C.c_int32),
        ("shape", C.c_int64 * TC_MAX_DIMS),
        ("stride", C.c_int64 * TC_MAX_DIMS),
    ]


class TcConvOpts(C.Structure):
    _fields_ = [
        ("method", C.c_int32),
        ("fft_threshold", C.c_int32),
        ("k_abs_sum", C.c_int64),
        ("k_host", C.c_void_p),
        ("workspace", C.c_void_p),
        ("workspace_bytes", C.c_size_t),
        ("band_rows", C.c_int32),
        ("reserved", C.c_int32),
    ]


class TcTuning(C.Structure):
    _fields_ = [("band_rows", C.c_int32), ("groups_per_cu", C.c_int32)]


class TcSeq(C.Structure):
    _fields_ = [
        ("frame0", C.c_void_p),
        ("frame_stride", C.c_int64),
        ("row_stride", C.c_int64),
        ("H", C.c_int32),
        ("W", C.c_int32),
        ("n_frames", C.c_int32),
        ("levels", C.c_int32),
    ]


# tc_ttc_level and tc_ttc_pick as numpy record types (same layout as the C structs)
LEVEL_DTYPE = np.dtype(
    [("sums", "<f8", (TC_NUM_SUMS,)), ("A", "<f8"), ("B", "<f8"), ("C", "<f8"), ("ttc", "<f8"), ("x0", "<f8"),
     ("y0", "<f8"), ("resid", "<f8"), ("n", "<i8"), ("level", "<i4"), ("status", "<i4")]
)
PICK_DTYPE = np.dtype(
    [("ttc", "<f8"), ("x0", "<f8"), ("y0", "<f8"), ("A", "<f8"), ("B", "<f8"), ("C", "<f8"), ("level", "<i4"),
     ("status", "<i4")]
)
assert LEVEL_DTYPE.itemsize == 152 and PICK_DTYPE.itemsize == 56

_P = C.c_void_p
_T = C.POINTER(TcTensor)
_I = C.c_int
_I32 = C.c_int32
_I64 = C.c_int64
_SZ = C.c_size_t

# name -> (restype, argtypes); every symbol declared in include/ttcconv.h
SIGNATURES = {
    "tc_status_str": (C.c_char_p, [_I]),
    "tc_version": (_I, []),
    "tc_device_check": (_I, [_I, C.POINTER(_I)]),
    "tc_conv_out_shape": (_I, [_T, _T, _I32, C.POINTER(_I64)]),
    "tc_conv_kernel_rank1": (_I, [C.POINTER(C.c_float), _I32, _I32, C.c_double, C.POINTER(C.c_float),
                                 C.POINTER(C.c_float)]),
    "tc_conv_nd_separable": (_I, [_T, _T, _T, _I32, _T, _P]),
    "tc_conv_nd": (_I, [_T, _T, _I32, _T, _P]),
    "tc_conv_workspace_size": (_I, [_T, _T, _I32, _I32, C.POINTER(_SZ)]),
    "tc_conv_nd_ex": (_I, [_T, _T, _I32, _T, C.POINTER(TcConvOpts), _P]),
    "tc_conv_fft_workspace_size": (_I, [_T, _T, _I32, C.POINTER(_SZ)]),
    "tc_conv_fft": (_I, [_T, _T, _I32, _T, _P, _SZ, _P]),
    "tc_conv2d_fft_workspace_size": (_I, [_T, _T, _I32, C.POINTER(_SZ)]),
    "tc_conv2d_fft": (_I, [_T, _T, _I32, _T, _P, _SZ, _P]),
    "tc_pyramid_shape": (_I, [_I64, _I64, _I32, C.POINTER(_I64), C.POINTER(_I64)]),
    "tc_image_pyramid": (_I, [_T, _I32, _T, _P]),
    "tc_horn_derivs": (_I, [_T, _T, _T, _T, _T, _P]),
    "tc_gradient": (_I, [_T, _I32, _T, _T, _T, _T, _P]),
    "tc_ttc_reselect": (_I, [_P, _I64, _I32, _I32, _P, _P]),
    "tc_ttc_plan_create": (_I, [C.POINTER(TcSeq), _I32, _I32, C.POINTER(_P)]),
    "tc_ttc_tuning_default": (_I, [_I32, _I32, C.POINTER(TcTuning)]),
    "tc_ttc_plan_create_ex": (_I, [C.POINTER(TcSeq), _I32, _I32, C.POINTER(TcTuning), C.POINTER(_P)]),
    "tc_ttc_plan_reset": (_I, [_P, C.POINTER(TcSeq), _I32]),
    "tc_ttc_plan_info": (_I, [_P, C.POINTER(_SZ), C.POINTER(_I64), C.POINTER(_I64)]),
    "tc_ttc_plan_upload": (_I, [_P, _P, _SZ, _P]),
    "tc_ttc_plan_run": (_I, [_P, _P, _SZ, _P, _P, _P]),
    "tc_ttc_plan_run_phase": (_I, [_P, _P, _SZ, _P, _P, _I32, _P]),
    "tc_ttc_plan_destroy": (None, [_P]),
    "tc_ttc_solve_batched": (_I, [C.POINTER(TcSeq), _I32, _I32, _P, _SZ, _P, _P, _P]),
    "tc_ttc_workspace_size": (_I, [_I64, _I64, _I32, C.POINTER(_SZ)]),
    "tc_ttc_variant_workspace_size": (_I, [_I64, _I64, _I32, _I32, _I32, C.POINTER(_SZ)]),
    "tc_ttc_solve_variant": (_I, [_T, _T, _I32, _I32, _I32, _P, _SZ, _P, _P, _P]),
    "tc_ttc_solve": (_I, [_T, _T, _I32, _P, _SZ, _P, _P, _P]),
    "tc_ttc_solve_noalloc": (_I, [_T, _T, _I32, _P, _P, _P]),
}

_lib = None


class TTCError(RuntimeError):
    def __init__(self, fn: str, code: int, lib=None):
        msg = lib.tc_status_str(code).decode() if lib is not None else str(code)
        super().__init__(f"{fn} failed: {msg} ({code})")
        self.code = code


def load(path: str = LIB_PATH):
    """Load libttcconv.so and declare every signature (raises if it is not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with `python -m paper_1612_08825_amd.build`")
    lib = C.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def check(fn: str, code: int):
    if code < 0:
        raise TTCError(fn, code, _lib)
    return code
