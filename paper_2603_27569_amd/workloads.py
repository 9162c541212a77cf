"""Seeded synthetic inputs shaped like the paper's workloads.

This module only draws inputs; it holds none of the transform's arithmetic.
Both the GPU tests and the FP64 checker consume the same complex64 arrays
produced here (values are drawn in FP64 with numpy's PCG64 and rounded once
to complex64).

The paper's workloads are batched SAR range/azimuth FFTs (Section II-D):
N = 2^10..2^14 with 256..16384 independent rows, and a 4096-bin x 256-line
block (Section VII-D).  No radar data is used; the recipes below stand in
for it:

  plain_uniform   N=256,  batch 64,  Re/Im i.i.d. U[-1, 1)          (seed 1001)
  plain_normal    N=4096, batch 256, Re/Im i.i.d. N(0, 1)           (seed 1002)
  chirp_noise     N=8192/16384, batch 1024: per row a linear-FM chirp of
                  length N/4 at a random offset, normalised bandwidth
                  U[0.2, 0.8], plus complex Gaussian noise at 10 dB SNR over
                  the chirp support                                   (seed 1003)
  spectral_energy N=4096, batch 512, x ~ N(0, 1); W ~ U[0, 1) float32  (1004/1104)
  ragged          2000 transforms, sizes 2^U{8..14}, N(0, 1) values   (seed 1005)
  to_storage      any of these rounded to a 16-bit storage format (IEEE
                  binary16 or bfloat16 pairs, nearest even) for the
                  half-storage path
  range_compression  N=4096, 256 lines: chirp_noise rows and a matched
                  filter given directly in frequency: unit-modulus quadratic
                  phase over the swept band, zero outside        (seed 1006)
"""
import numpy as np

SIZES = tuple(1 << e for e in range(8, 15))


def rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def _to_c64(re, im):
    out = np.empty(re.shape, dtype=np.complex64)
    out.real = re
    out.imag = im
    return out


def complex_uniform(shape, seed):
    g = rng(seed)
    re = g.uniform(-1.0, 1.0, size=shape)
    im = g.uniform(-1.0, 1.0, size=shape)
    return _to_c64(re, im)


def complex_normal(shape, seed):
    g = rng(seed)
    re = g.standard_normal(size=shape)
    im = g.standard_normal(size=shape)
    return _to_c64(re, im)


def plain_uniform(n=256, batch=64, seed=1001):
    return complex_uniform((batch, n), seed)


def plain_normal(n=4096, batch=256, seed=1002):
    return complex_normal((batch, n), seed)


def delta_batch(n, batch):
    """Row b is a unit impulse at position b mod n."""
    x = np.zeros((batch, n), dtype=np.complex64)
    x[np.arange(batch), np.arange(batch) % n] = 1.0
    return x


def tone_bins(n, batch):
    return (37 * np.arange(batch, dtype=np.int64) + 5) % n


def tone_batch(n, batch):
    """Row b is exp(+2 pi i k_b m / n), k_b = (37 b + 5) mod n.

    The phase k_b * m is reduced mod n in integers before the FP64 cos/sin,
    then rounded once to complex64."""
    k = tone_bins(n, batch)[:, None]
    m = np.arange(n, dtype=np.int64)[None, :]
    ph = 2.0 * np.pi * ((k * m) % n).astype(np.float64) / n
    return _to_c64(np.cos(ph), np.sin(ph))


def chirp_noise(n, batch=1024, seed=1003, snr_db=10.0):
    """Linear-FM chirp of length L = n/4 at offset o ~ U{0..n-L}, sweeping
    -beta/2 .. +beta/2 cycles/sample with beta ~ U[0.2, 0.8], plus complex
    Gaussian noise of variance 10^(-snr_db/10) on every sample (SNR taken
    over the chirp support, where the chirp has unit power).

    Returns (x complex64 [batch, n], meta dict)."""
    g = rng(seed)
    L = n // 4
    offs = g.integers(0, n - L + 1, size=batch)
    beta = g.uniform(0.2, 0.8, size=batch)
    sigma2 = 10.0 ** (-snr_db / 10.0)
    sd = np.sqrt(sigma2 / 2.0)
    nre = g.standard_normal(size=(batch, n)) * sd
    nim = g.standard_normal(size=(batch, n)) * sd
    m = np.arange(L, dtype=np.float64)[None, :]
    phase = -0.5 * beta[:, None] * m + beta[:, None] / (2.0 * L) * m * m
    ph = 2.0 * np.pi * np.mod(phase, 1.0)
    re = nre.copy()
    im = nim.copy()
    cols = offs[:, None] + np.arange(L)[None, :]
    rows = np.arange(batch)[:, None]
    re[rows, cols] += np.cos(ph)
    im[rows, cols] += np.sin(ph)
    meta = {"chirp_len": L, "offsets": offs, "beta": beta, "noise_var": sigma2,
            "snr_reading": "over chirp support (unit power)"}
    return _to_c64(re, im), meta


def spectral_energy_inputs(n=4096, batch=512, seed=1004, wseed=1104):
    x = complex_normal((batch, n), seed)
    w = rng(wseed).uniform(0.0, 1.0, size=n).astype(np.float32)
    return x, w


def ragged_sizes(count=2000, seed=1005):
    g = rng(seed)
    e = g.integers(8, 15, size=count)
    return (np.int64(1) << e).astype(np.int64)


def ragged(count=2000, seed=1005):
    """Returns (sizes int64[count], offsets int64[count], packed complex64).

    Sizes are 2^e with e ~ U{8..14}; rows are packed in draw order at the
    exclusive prefix sum of the sizes; values are i.i.d. N(0, 1)."""
    sizes = ragged_sizes(count, seed)
    offsets = np.zeros(count, dtype=np.int64)
    if count > 1:
        offsets[1:] = np.cumsum(sizes)[:-1]
    total = int(sizes.sum())
    data = complex_normal((total,), seed + 7919)
    return sizes, offsets, data


def range_compression_inputs(n=4096, batch=256, seed=1006, beta=0.5):
    """SAR range-compression block (4096 bins x 256 lines): rows from
    chirp_noise and a filter spectrum h of length n.  h is the stationary-phase
    form of a linear-FM chirp spectrum, written down directly: for frequency
    bins f = k/n (centred, in cycles/sample) inside the band |f| < beta/2,
    h[k] = exp(i*pi*L*f^2/beta) with L = n/4, else 0.

    Returns (x complex64 [batch, n], h complex64 [n])."""
    x, _ = chirp_noise(n, batch, seed)
    k = np.arange(n, dtype=np.float64)
    f = np.where(k < n / 2, k, k - n) / n
    L = n // 4
    ph = np.pi * L * f * f / beta
    inband = np.abs(f) < beta / 2
    re = np.where(inband, np.cos(ph), 0.0)
    im = np.where(inband, np.sin(ph), 0.0)
    return x, _to_c64(re, im)


def bf16_bits(a):
    """float32 -> bfloat16 bit patterns (uint16), rounding to nearest even."""
    u = np.ascontiguousarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16).astype(np.uint16)
    nan = np.isnan(np.asarray(a, dtype=np.float32))
    r[nan] = ((u[nan] >> 16) | 0x40).astype(np.uint16)
    return r


def bf16_value(bits):
    """bfloat16 bit patterns -> float32 values (exact)."""
    return (np.asarray(bits, dtype=np.uint16).astype(np.uint32) << 16).view(np.float32)


def to_storage(x, fmt):
    """Round complex values to a 16-bit storage format.

    Returns (stored, values): `stored` is an array of shape x.shape + (2,)
    holding (real, imaginary) as float16 (fmt "f16") or as bfloat16 bit
    patterns in uint16 (fmt "bf16"); `values` is complex128, the exact values
    those hold (what the transform is then applied to)."""
    x = np.asarray(x)
    pair = np.stack([x.real, x.imag], axis=-1).astype(np.float32)
    if fmt == "f16":
        stored = pair.astype(np.float16)
        back = stored.astype(np.float64)
    elif fmt == "bf16":
        stored = bf16_bits(pair)
        back = bf16_value(stored).astype(np.float64)
    else:
        raise ValueError("fmt must be 'f16' or 'bf16'")
    return stored, back[..., 0] + 1j * back[..., 1]
