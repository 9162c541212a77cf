"""ctypes declarations of libstockfft.so (include/stockfft.h).

Argument marshalling only: every entry point here forwards to the C ABI.
The library must be built in-tree (``python paper_2603_27569_amd/build.py``
or ``__graft_entry__.build()``); importing a function that needs it raises
when it is missing -- there is no fallback implementation.
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libstockfft.so")

FFT_FORWARD = -1
FFT_BACKWARD = 1
FFT_ALGO_AUTO = 0
FFT_ALGO_SINGLE_PASS = 1
FFT_ALGO_FOUR_STEP = 2
FFT_IO_C64 = 0
FFT_IO_C16 = 1
FFT_IO_BC16 = 2
FFT_IO_C16_MMA = 3
FFT_IO_BC16_MMA = 4

STATUS = {
    0: "FFT_SUCCESS", 1: "FFT_INVALID_SIZE", 2: "FFT_INVALID_BATCH",
    3: "FFT_INVALID_DIRECTION", 4: "FFT_INVALID_POINTER", 5: "FFT_MISALIGNED",
    6: "FFT_OVERLAP", 7: "FFT_INVALID_PLAN", 8: "FFT_NO_DEVICE",
    9: "FFT_ALLOC_FAILED", 10: "FFT_HIP_ERROR", 11: "FFT_INVALID_ARGUMENT",
    12: "FFT_UNSUPPORTED",
}
CODES = {v: k for k, v in STATUS.items()}

# Every symbol include/stockfft.h declares, with its ctypes signature.
_vp = ctypes.c_void_p
_i64 = ctypes.c_int64
_int = ctypes.c_int
_pvp = ctypes.POINTER(ctypes.c_void_p)
SIGNATURES = {
    "fft_plan": (_int, [_pvp, _i64, _i64, _int]),
    "fft_plan_config": (_int, [_pvp, _i64, _i64, _int, _int, ctypes.c_char_p]),
    "fft_exec": (_int, [_vp, _vp, _vp, _vp]),
    "fft_destroy": (_int, [_vp]),
    "fft_exec_spectral_energy": (_int, [_vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    "fft_exec_spectral_energy_noalloc": (_int, [_vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    "fft_exec_matched_filter": (_int, [_vp, _vp, _vp, _vp, _vp]),
    "fft_plan_ragged": (_int, [_pvp, ctypes.POINTER(_i64), _i64, _int]),
    "fft_exec_ragged": (_int, [_vp, _vp, _vp, _vp]),
    "fft_exec_io": (_int, [_vp, _vp, _vp, ctypes.c_int, _vp]),
    "fft_exec_ragged_direct": (_int, [_vp, _vp, _vp, _vp]),
    "fft_exec_ragged_plain": (_int, [_vp, _pvp, _pvp, _vp]),
    "fft_destroy_ragged": (_int, [_vp]),
    "fft_ragged_shapes": (_int, [_i64, ctypes.c_char_p, _i64]),
    "fft_tune_set_ragged": (_int, [_i64, ctypes.c_char_p]),
    "fft_tune_query_ragged": (_int, [_i64, ctypes.c_char_p, _i64]),
    "fft_tune_query_filter": (_int, [_i64, _i64, ctypes.c_char_p, _i64]),
    "fft_tune_query_fused": (_int, [_i64, _i64, ctypes.c_char_p, _i64]),
    "fft_tune_query_storage16": (_int, [_i64, _i64, ctypes.c_char_p, _i64]),
    "fft_tune_clear_ragged": (_int, []),
    "fft_tune_load": (_int, [ctypes.c_char_p]),
    "fft_tune_set": (_int, [_i64, _i64, _i64, ctypes.c_char_p]),
    "fft_tune_clear": (_int, []),
    "fft_tune_query": (_int, [_i64, _i64, ctypes.c_char_p, _i64]),
    "fft_set_launch_limit": (_int, [_i64]),
    "fft_variant_count": (_int, []),
    "fft_variant_describe": (_int, [_int, ctypes.c_char_p, _i64]),
    "fft_variant_twiddles": (_int, [_int, ctypes.POINTER(ctypes.c_float), _i64, ctypes.POINTER(_i64)]),
    "fft_plan_describe": (_int, [_vp, ctypes.c_char_p, _i64]),
    "fft_status_string": (ctypes.c_char_p, [_int]),
    "fft_last_hip_error": (_int, []),
    "fft_version": (_int, []),
}

_lib = None


class StockfftError(RuntimeError):
    def __init__(self, func, status):
        self.status = status
        self.name = STATUS.get(status, str(status))
        msg = f"{func} failed: {self.name}"
        if _lib is not None:
            msg += f" ({_lib.fft_status_string(status).decode()})"
            if status == CODES["FFT_HIP_ERROR"]:
                msg += f", hipError {_lib.fft_last_hip_error()}"
        super().__init__(msg)


def lib():
    """Load libstockfft.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(
            f"{LIB_PATH} is missing: build the HIP library first "
            "(python paper_2603_27569_amd/build.py)")
    L = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def check(func, status):
    if status != 0:
        raise StockfftError(func, status)
    return status
