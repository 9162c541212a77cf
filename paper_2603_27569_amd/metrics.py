"""Accuracy gates and throughput conventions.

Throughput follows the paper's convention (Section VI-A): an N-point complex
transform counts 5 N log2 N floating-point operations; GFLOPS is that count
times the batch divided by the time.  Algorithmic HBM traffic of one
out-of-place transform is 16 N bytes (read 8N, write 8N, complex64).
"""
import math

import numpy as np

HBM_PEAK_GBS = 8000.0


def fft_flops(n, batch=1):
    return 5.0 * n * math.log2(n) * batch


def fft_bytes(n, batch=1):
    return 16.0 * n * batch


def gflops(n, batch, seconds):
    return fft_flops(n, batch) / seconds / 1e9


def per_row_errors(y, ref, x):
    """Return (rel_rms[b], max_abs[b], x_norm[b]) over rows of complex arrays.

    rel_rms_b = ||y_b - X_b||_2 / ||X_b||_2; max_abs_b = max_k |y_b - X_b|;
    the max-abs gate is taken relative to the input row norm ||x_b||_2."""
    y = np.asarray(y).reshape(-1, np.asarray(y).shape[-1]).astype(np.complex128)
    ref = np.asarray(ref).reshape(y.shape).astype(np.complex128)
    x = np.asarray(x).reshape(-1, np.asarray(x).shape[-1]).astype(np.complex128)
    d = y - ref
    num = np.sqrt(np.sum(np.abs(d) ** 2, axis=1))
    den = np.sqrt(np.sum(np.abs(ref) ** 2, axis=1))
    with np.errstate(divide="ignore", invalid="ignore"):
        rel = np.where(den > 0, num / den, np.where(num == 0, 0.0, np.inf))
    mabs = np.max(np.abs(d), axis=1) if d.shape[1] else np.zeros(d.shape[0])
    xn = np.sqrt(np.sum(np.abs(x) ** 2, axis=1))
    return rel, mabs, xn


REL_RMS_GATE = 5e-6
MAX_ABS_GATE = 1e-5  # times the input row norm, for N <= 16384


def max_abs_gate(n):
    """The max-abs tolerance (times ||x_b||_2) for length n.

    1e-5 up to N = 16384, the paper's range.  Above it an output bin can
    reach sqrt(N) ||x_b||_2 (Cauchy-Schwarz), and one unit in the last place
    of such a bin, 2^-23 sqrt(N) ||x_b||_2, exceeds 1e-5 ||x_b||_2 from
    N = 32768 on; there the gate is two such units, 2^-22 sqrt(N)."""
    if n <= 16384:
        return MAX_ABS_GATE
    return 2.0 ** -22 * float(n) ** 0.5


def gate(y, ref, x, rel_gate=REL_RMS_GATE, abs_gate=None):
    """Return (ok, worst_rel_rms, median_rel_rms, worst_abs_ratio).  abs_gate
    defaults to max_abs_gate(N) for the rows' length N."""
    if abs_gate is None:
        abs_gate = max_abs_gate(np.asarray(y).shape[-1])
    rel, mabs, xn = per_row_errors(y, ref, x)
    with np.errstate(divide="ignore", invalid="ignore"):
        ratio = np.where(xn > 0, mabs / xn, np.where(mabs == 0, 0.0, np.inf))
    ok = bool(np.all(rel <= rel_gate) and np.all(ratio <= abs_gate))
    return ok, float(rel.max(initial=0.0)), float(np.median(rel) if rel.size else 0.0), \
        float(ratio.max(initial=0.0))


GRAD_REL_GATE = 1e-4


def grad_gate(g, ref, rel_gate=GRAD_REL_GATE):
    """Gradient gate, row by row: every row b must satisfy
    ||g_b - ref_b||_2 / ||ref_b||_2 <= rel_gate (1e-4 against the analytic
    FP64 F^H g), and the rows must also pass the transform gate of `gate`
    taken against the reference gradient itself (rel-RMS <= 5e-6 and max-abs
    <= 1e-5 ||ref_b||_2), since the gradient is two FP32 transforms deep.
    A row whose reference is exactly zero must come out exactly zero.
    Returns (ok, worst_row_rel, worst_abs_ratio)."""
    rel, _, _ = per_row_errors(g, ref, ref)
    ok_t, _, _, ab = gate(g, ref, ref)
    ok = bool(np.all(rel <= rel_gate) and ok_t)
    return ok, float(rel.max(initial=0.0)), float(ab)


# 16-bit storage: unit roundoff of one rounding to the format.
STORAGE_UNIT_ROUNDOFF = {"f16": 2.0 ** -11, "bf16": 2.0 ** -8}


def dft16_matrix_error(fmt):
    """||M_fmt - M||_2 / 4 for the real 32 x 32 form M = [[C, S], [-S, C]] of
    the 16-point DFT (C, S: cos and sin of 2 pi k r / 16) rounded entrywise to
    the 16-bit format: the relative error one pass of matrix-core DFTs takes
    from its rounded matrix (M / 4 is orthogonal)."""
    k = np.arange(16)
    ang = 2.0 * np.pi * np.outer(k, k) / 16.0
    c, s = np.cos(ang), np.sin(ang)
    m = np.block([[c, s], [-s, c]])
    if fmt == "f16":
        mr = m.astype(np.float16).astype(np.float64)
    else:
        from .workloads import bf16_bits, bf16_value
        mr = bf16_value(bf16_bits(m.astype(np.float32))).astype(np.float64)
    return float(np.linalg.norm(mr - m, 2) / 4.0)


def mma_passes(n):
    """(radix-16 passes on the matrix cores, all passes) of the matrix-core
    path at length n = 16^P RL (RL = 1, 2, 4 or 8: one more pass on the
    vector ALUs when RL > 1)."""
    p, m = 0, n
    while m % 16 == 0 and m >= 16:
        m //= 16
        p += 1
    return p, p + (1 if m > 1 else 0)


def mma_gate_factor(fmt, passes=3, matrix_passes=None):
    """Error factor g (in units of u) for the matrix-core 16-bit path: the
    inputs of each of the `passes` passes and the output are each rounded at
    most once (relative RMS <= u / sqrt(3) each, independent, so
    sqrt(passes + 1) u / sqrt(3) together), and every radix-16 pass
    (`matrix_passes`, default all) adds the rounded matrix's error (linearly,
    as it is systematic)."""
    u = STORAGE_UNIT_ROUNDOFF[fmt]
    mp = passes if matrix_passes is None else matrix_passes
    return float(np.sqrt((passes + 1) / 3.0) + mp * dft16_matrix_error(fmt) / u)


def gate_storage(y, ref, x, fmt, mma=False):
    """Gate for results stored in a 16-bit format (`ref` is the exact DFT of
    the values actually stored as input).  One rounding of the output to a
    format with unit roundoff u leaves a relative error of at most u per bin
    and about u / sqrt(3) in RMS, so: rel-RMS <= u, and per bin
    |y - X| <= u |X|max + 1e-5 ||x_b||_2 (the FP32 arithmetic's own share, as
    in the FP32 gate).  With mma=True (16-point DFTs on the matrix cores,
    mma_gate_factor for the row length's passes) the RMS bound is g u and the
    per-bin one 2 g u |X|max +
    1e-5 ||x_b||_2 (a bin's error is the largest of n samples where the RMS
    averages them).  Returns (ok, worst_rel_rms, median_rel_rms,
    worst_abs_ratio) with the abs ratio taken against that bound."""
    u = STORAGE_UNIT_ROUNDOFF[fmt]
    rel, mabs, xn = per_row_errors(y, ref, x)
    r = np.asarray(ref).reshape(rel.shape[0], -1)
    g = 1.0
    if mma:
        p16, ptot = mma_passes(r.shape[1])
        g = mma_gate_factor(fmt, ptot, p16)
    bound = (2.0 * g if mma else 1.0) * u * np.max(np.abs(r), axis=1) + 1e-5 * xn
    with np.errstate(divide="ignore", invalid="ignore"):
        ratio = np.where(bound > 0, mabs / bound, np.where(mabs == 0, 0.0, np.inf))
    ok = bool(np.all(rel <= g * u) and np.all(ratio <= 1.0))
    return ok, float(rel.max(initial=0.0)), float(np.median(rel) if rel.size else 0.0), \
        float(ratio.max(initial=0.0))
