"""ctypes declarations of libstockref.so (include/stockref.h): measurement
references beside the transform library -- an empty kernel, copies in the
transform's launch shape and in a wide grid, the middle steps of the two
unfused chains, and the single-pass transform with phase stamps.

Argument marshalling only.  The library must be built in-tree
(``python paper_2603_27569_amd/build.py``); loading it raises when it is
missing.
"""
import ctypes
import os

from ._lib import STATUS, StockfftError

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libstockref.so")

_vp = ctypes.c_void_p
_i64 = ctypes.c_int64
_int = ctypes.c_int
SIGNATURES = {
    "ref_empty": (_int, [_i64, _int, _vp]),
    "ref_copy_rows": (_int, [_vp, _vp, _i64, _i64, _int, _vp]),
    "ref_copy_wide": (_int, [_vp, _vp, _i64, _vp]),
    "ref_lds_exchange": (_int, [_i64, ctypes.c_int, _vp, _vp]),
    "ref_weight_energy": (_int, [_vp, _vp, _vp, _i64, _i64, _vp]),
    "ref_filter_multiply": (_int, [_vp, _vp, _i64, _i64, _vp]),
    "ref_timeline": (_int, [ctypes.c_char_p, _vp, _vp, _vp, _i64, _int, _vp, _vp]),
    "ref_timeline_variants": (_int, [ctypes.c_char_p, _i64]),
    "ref_last_hip_error": (_int, []),
}

_lib = None


def lib():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it first "
                           "(python paper_2603_27569_amd/build.py)")
    L = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def _check(func, status):
    if status != 0:
        raise StockfftError(func, status)


def _p(x):
    return _vp(int(x) if x else 0)


def empty(groups, threads, stream=0):
    _check("ref_empty", lib().ref_empty(int(groups), int(threads), _p(stream)))


def copy_rows(src, dst, n, batch, lanes, stream=0):
    _check("ref_copy_rows", lib().ref_copy_rows(_p(src), _p(dst), int(n), int(batch), int(lanes),
                                                _p(stream)))


def copy_wide(src, dst, nbytes, stream=0):
    _check("ref_copy_wide", lib().ref_copy_wide(_p(src), _p(dst), int(nbytes), _p(stream)))


def lds_exchange(groups, rounds, out, stream=0):
    _check("ref_lds_exchange", lib().ref_lds_exchange(int(groups), int(rounds), _p(out), _p(stream)))


def weight_energy(y, w, row_loss, n, batch, stream=0):
    _check("ref_weight_energy", lib().ref_weight_energy(_p(y), _p(w), _p(row_loss), int(n),
                                                        int(batch), _p(stream)))


def filter_multiply(y, h, n, batch, stream=0):
    _check("ref_filter_multiply", lib().ref_filter_multiply(_p(y), _p(h), int(n), int(batch),
                                                            _p(stream)))


def timeline_variants():
    buf = ctypes.create_string_buffer(1024)
    _check("ref_timeline_variants", lib().ref_timeline_variants(buf, len(buf)))
    return buf.value.decode().split(",")


def timeline(variant, src, dst, tw, batch, inverse, stamps, stream=0):
    _check("ref_timeline", lib().ref_timeline(variant.encode(), _p(src), _p(dst), _p(tw),
                                              int(batch), 1 if inverse else 0, _p(stamps),
                                              _p(stream)))


def status_name(code):
    return STATUS.get(code, str(code))
