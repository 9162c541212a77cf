"""The oracle's pins must catch plausible mistakes.

Each case below plants one mistake (a flipped sign, a dropped factor, a
wrong index or exponent, a missing conjugate) in a copy of the oracle's
source, builds that copy on the CPU, and checks that at least one of the
independent pins (closed forms, numpy cross-check, exact central differences,
special cases) rejects it.  The unmodified source must pass them all.
"""
import ctypes
import os

import numpy as np
import pytest

from oracle import build as obuild

SRC = open(obuild.SRC).read()

MUTATIONS = {
    "root_sign": ("*im = (double)sign * sin(ang);", "*im = -(double)sign * sin(ang);"),
    "combine_sign": ("out[2 * (h + k)] = er - tr;", "out[2 * (h + k)] = er + tr;"),
    "twiddle_exponent": ("unit_root(k, n, sign, &wr, &wi);", "unit_root(k, h, sign, &wr, &wi);"),
    "twiddle_dropped": ("double tr = wr * orr - wi * oi;", "double tr = orr;"),
    "direct_exponent": ("int64_t m = (j * k) % n;", "int64_t m = (j + k) % n;"),
    "direct_conj_term": ("si += xr * wi + xi * wr;", "si += xr * wi - xi * wr;"),
    "odd_half_offset": ("fft_recursive(x + 2 * xs, 2 * xs, out + 2 * h, h, sign, roots);",
                        "fft_recursive(x, 2 * xs, out + 2 * h, h, sign, roots);"),
    "grad_factor_two": ("yb[2 * k] = 2.0 * w2 * yr;", "yb[2 * k] = w2 * yr;"),
    "loss_w_not_squared": ("acc += w2 * (yr * yr + yi * yi);", "acc += w[k] * (yr * yr + yi * yi);"),
    "grad_wrong_direction": ("fft_recursive(yb, 1, grad + 2 * b * n, n, +1, roots);",
                             "fft_recursive(yb, 1, grad + 2 * b * n, n, -1, roots);"),
    "mf_missing_conj": ("double hr = h[2 * k], hi = -h[2 * k + 1];",
                        "double hr = h[2 * k], hi = h[2 * k + 1];"),
    "mf_missing_scale": ("for (int64_t k = 0; k < 2 * n; ++k) ob[k] /= (double)n;",
                         "for (int64_t k = 0; k < 2 * n; ++k) ob[k] /= 1.0;"),
}


class _Lib:
    def __init__(self, path):
        lib = ctypes.CDLL(path)
        dp = ctypes.POINTER(ctypes.c_double)
        i64 = ctypes.c_int64
        for name in ("oracle_dft_direct", "oracle_fft"):
            getattr(lib, name).argtypes = [dp, dp, i64, i64, ctypes.c_int]
        lib.oracle_spectral_energy.argtypes = [dp, dp, i64, i64, dp, dp]
        lib.oracle_matched_filter.argtypes = [dp, dp, i64, i64, dp]
        self.lib = lib

    @staticmethod
    def _p(a):
        return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))

    def tr(self, name, x, sign):
        x = np.ascontiguousarray(x, dtype=np.complex128).reshape(-1, x.shape[-1])
        y = np.empty_like(x)
        getattr(self.lib, name)(self._p(x), self._p(y), x.shape[1], x.shape[0], sign)
        return y

    def se(self, x, w):
        x = np.ascontiguousarray(x, dtype=np.complex128).reshape(-1, x.shape[-1])
        w = np.ascontiguousarray(w, dtype=np.float64)
        loss = np.empty(x.shape[0])
        g = np.empty_like(x)
        self.lib.oracle_spectral_energy(self._p(x), self._p(w), x.shape[1], x.shape[0],
                                        self._p(loss), self._p(g))
        return loss, g

    def mf(self, x, h):
        x = np.ascontiguousarray(x, dtype=np.complex128).reshape(-1, x.shape[-1])
        h = np.ascontiguousarray(h, dtype=np.complex128)
        out = np.empty_like(x)
        self.lib.oracle_matched_filter(self._p(x), self._p(h), x.shape[1], x.shape[0], self._p(out))
        return out


def _pins_pass(L):
    """A compact subset of the oracle pins; True iff every one holds."""
    g = np.random.default_rng(5)
    ok = True

    def close(a, b, tol=1e-10):
        return float(np.max(np.abs(a - b))) <= tol * max(1.0, float(np.max(np.abs(b))))

    for n in (8, 16, 256, 1024):
        for name in ("oracle_dft_direct", "oracle_fft"):
            x = g.standard_normal((2, n)) + 1j * g.standard_normal((2, n))
            ok &= close(L.tr(name, x, -1), np.fft.fft(x, axis=-1))
            ok &= close(L.tr(name, x, +1), np.fft.ifft(x, axis=-1) * n)
    n = 128
    x = g.standard_normal((2, n)) + 1j * g.standard_normal((2, n))
    w = g.uniform(0, 1, n)
    loss, grad = L.se(x, w)
    ok &= close(loss, np.sum(w ** 2 * np.abs(np.fft.fft(x, axis=-1)) ** 2, axis=1))
    for i in (3, 77, 200):
        for comp in (1.0, 1j):
            e = np.zeros(x.size, complex)
            e[i] = comp
            e = e.reshape(x.shape)
            fd = (np.sum(L.se(x + e, w)[0]) - np.sum(L.se(x - e, w)[0])) / 2.0
            got = grad.reshape(-1)[i]
            got = got.real if comp == 1.0 else got.imag
            ok &= abs(fd - got) <= 1e-8 * max(1.0, float(np.max(np.abs(grad))))
    s = 11
    k = np.arange(n)
    h = np.exp(-2j * np.pi * ((s * k) % n) / n)
    ok &= close(L.mf(x, h), np.roll(x, -s, axis=-1))
    return bool(ok)


def _build_variant(tmp_path, name, text):
    src = tmp_path / f"{name}.c"
    src.write_text(text)
    out = str(tmp_path / f"lib{name}.so")
    obuild.build(out=out, src=str(src))
    return _Lib(out)


def test_unmodified_oracle_passes_pins(tmp_path):
    assert _pins_pass(_build_variant(tmp_path, "clean", SRC))


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_planted_mistake_is_caught(tmp_path, name):
    old, new = MUTATIONS[name]
    assert SRC.count(old) == 1, f"mutation anchor for {name} not unique in the oracle source"
    lib = _build_variant(tmp_path, name, SRC.replace(old, new))
    assert not _pins_pass(lib), f"planted mistake {name} was not caught by the pins"
