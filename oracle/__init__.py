"""FP64 CPU oracle for the batched complex DFT -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The GPU library never loads it and
shares no code with it.

Everything is computed in FP64 from the DFT definition (the paper, Section
II-A): X[k] = sum_n x[n] exp(sign 2 pi i n k / N), sign = -1 forward,
+1 backward, no scaling.  Inputs that were complex64 are promoted exactly
to complex128, so the oracle sees the very values the GPU sees.
"""
import ctypes
import os

import numpy as np

from . import build as _build

_lib = None


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_build.LIB) or (
            os.path.getmtime(_build.LIB) < os.path.getmtime(_build.SRC)):
        _build.build()
    lib = ctypes.CDLL(_build.LIB)
    dp = ctypes.POINTER(ctypes.c_double)
    i64 = ctypes.c_int64
    for name in ("oracle_dft_direct", "oracle_fft"):
        f = getattr(lib, name)
        f.argtypes = [dp, dp, i64, i64, ctypes.c_int]
        f.restype = ctypes.c_int
    lib.oracle_spectral_energy.argtypes = [dp, dp, i64, i64, dp, dp]
    lib.oracle_spectral_energy.restype = ctypes.c_int
    lib.oracle_matched_filter.argtypes = [dp, dp, i64, i64, dp]
    lib.oracle_matched_filter.restype = ctypes.c_int
    lib.oracle_max_threads.restype = ctypes.c_int
    lib.oracle_set_threads.argtypes = [ctypes.c_int]
    _lib = lib
    return lib


def _as_c128(x):
    a = np.ascontiguousarray(np.asarray(x), dtype=np.complex128)
    return a


def _ptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _rows(a):
    if a.ndim == 1:
        return a.reshape(1, -1)
    return a.reshape(-1, a.shape[-1])


def _transform(fn_name, x, inverse):
    a = _as_c128(x)
    shape = a.shape
    rows = _rows(a)
    n = rows.shape[1]
    out = np.empty_like(rows)
    rc = getattr(_load(), fn_name)(_ptr(rows), _ptr(out), n, rows.shape[0],
                                   1 if inverse else -1)
    if rc != 0:
        raise ValueError(f"{fn_name} failed with code {rc} (n={n})")
    return out.reshape(shape)


def dft(x, inverse=False):
    """Direct O(N^2) DFT along the last axis (any N >= 1), unscaled."""
    return _transform("oracle_dft_direct", x, inverse)


def fft(x, inverse=False):
    """Recursive radix-2 FFT along the last axis (N a power of two or N <= 64),
    unscaled in both directions."""
    return _transform("oracle_fft", x, inverse)


def spectral_energy(x, w):
    """Return (row_loss, grad) for L = sum_b sum_k w_k^2 |(F x_b)[k]|^2.

    row_loss has one FP64 value per row; grad = F^H (2 w^2 * F x_b) per row,
    which is dL/dRe(x) + i dL/dIm(x)."""
    a = _as_c128(x)
    rows = _rows(a)
    n = rows.shape[1]
    wv = np.ascontiguousarray(np.asarray(w, dtype=np.float64).reshape(-1))
    if wv.shape[0] != n:
        raise ValueError("w must have length N")
    loss = np.empty(rows.shape[0], dtype=np.float64)
    grad = np.empty_like(rows)
    rc = _load().oracle_spectral_energy(_ptr(rows), _ptr(wv), n, rows.shape[0],
                                        _ptr(loss), _ptr(grad))
    if rc != 0:
        raise ValueError(f"oracle_spectral_energy failed with code {rc}")
    return loss, grad.reshape(a.shape)


def matched_filter(x, h):
    """out_b = F^{-1}(conj(h) * F x_b) with F^{-1} = backward / N."""
    a = _as_c128(x)
    rows = _rows(a)
    n = rows.shape[1]
    hv = _as_c128(h).reshape(-1)
    if hv.shape[0] != n:
        raise ValueError("h must have length N")
    out = np.empty_like(rows)
    rc = _load().oracle_matched_filter(_ptr(rows), _ptr(hv), n, rows.shape[0], _ptr(out))
    if rc != 0:
        raise ValueError(f"oracle_matched_filter failed with code {rc}")
    return out.reshape(a.shape)


def max_threads():
    return int(_load().oracle_max_threads())


def set_threads(t):
    _load().oracle_set_threads(int(t))
