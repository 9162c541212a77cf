"""Host-side checks: the throughput convention against the paper's printed
numbers, and the seeded workload generators."""
import json
import os

import numpy as np
import pytest

from paper_2603_27569_amd import metrics, workloads

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_tables.json")


def _golden():
    with open(GOLDEN) as f:
        return json.load(f)


def test_flop_convention_matches_table_vi():
    """Table VI's GFLOPS and us/FFT columns agree under 5 N log2 N."""
    for row in _golden()["table_vi_n4096_batch256"]["rows"]:
        g = metrics.gflops(4096, 1, row["us_per_fft"] * 1e-6)
        assert abs(g - row["gflops"]) / row["gflops"] < 0.005, row


def test_bmax_equation():
    b = _golden()["bmax"]
    assert b["local_mem_bytes"] // b["bytes_per_elem"] == b["bmax"] == 4096


def test_bytes_convention():
    assert metrics.fft_bytes(4096, 256) == 16 * 1024 * 1024
    assert metrics.fft_flops(4096, 256) == 62914560


def test_max_abs_gate_by_length():
    for n in (256, 4096, 16384):
        assert metrics.max_abs_gate(n) == 1e-5
    for e in range(15, 21):
        n = 2 ** e
        # two units in the last place of the largest bin sqrt(N) ||x|| can give
        assert metrics.max_abs_gate(n) == 2.0 ** -22 * 2.0 ** (e / 2)
        assert metrics.max_abs_gate(n) > 1e-5
    # a length-2^20 tone: the peak bin N ||x|| / sqrt(N) off by one ulp passes
    n = 2 ** 20
    x = np.exp(2j * np.pi * 3 * np.arange(n) / n)[None, :]
    ref = np.zeros_like(x)
    ref[0, 3] = n
    y = ref.copy()
    y[0, 3] += np.spacing(np.float32(n))
    assert metrics.gate(y, ref, x)[0]
    y[0, 3] += 4 * np.spacing(np.float32(n))
    assert not metrics.gate(y, ref, x)[0]


def test_gate_logic():
    x = workloads.plain_normal(64, 4, seed=3).astype(np.complex128)
    ok, worst, med, ab = metrics.gate(x, x, x)
    assert ok and worst == 0.0 and ab == 0.0
    y = x.copy()
    y[1, 3] += 1e-3
    ok, worst, _, _ = metrics.gate(y, x, x)
    assert not ok and worst > 5e-6
    z = np.zeros((2, 8), complex)
    assert metrics.gate(z, z, z)[0]
    z2 = z.copy()
    z2[0, 0] = 1e-30
    assert not metrics.gate(z2, z, z)[0]


def test_generators_deterministic_and_typed():
    a = workloads.plain_normal()
    b = workloads.plain_normal()
    assert a.dtype == np.complex64 and a.shape == (256, 4096)
    assert np.array_equal(a, b)
    assert not np.array_equal(a, workloads.plain_normal(seed=1))
    u = workloads.plain_uniform()
    assert u.shape == (64, 256)
    assert np.all(np.abs(u.real) <= 1) and np.all(np.abs(u.imag) <= 1)
    assert abs(np.mean(a.real)) < 0.01 and abs(np.std(a.real) - 1) < 0.01


def test_delta_and_tone():
    d = workloads.delta_batch(256, 300)
    assert np.all(np.sum(d != 0, axis=1) == 1)
    assert d[299, 299 % 256] == 1
    t = workloads.tone_batch(256, 8)
    assert np.allclose(np.abs(t), 1.0, atol=1e-6)
    k = workloads.tone_bins(256, 8)
    m = np.arange(256)
    ref = np.exp(2j * np.pi * k[3] * m / 256)
    assert np.max(np.abs(t[3] - ref)) < 1e-6


@pytest.mark.parametrize("n", [8192, 16384])
def test_chirp_noise_statistics(n):
    x, meta = workloads.chirp_noise(n, batch=64)
    assert x.shape == (64, n) and x.dtype == np.complex64
    L = meta["chirp_len"]
    assert L == n // 4
    offs = meta["offsets"]
    assert np.all(offs >= 0) and np.all(offs + L <= n)
    assert np.all((meta["beta"] >= 0.2) & (meta["beta"] <= 0.8))
    # Off-support power is the noise variance (0.1 at 10 dB over the chirp power 1).
    off = []
    on = []
    for b in range(64):
        mask = np.zeros(n, bool)
        mask[offs[b]:offs[b] + L] = True
        off.append(np.mean(np.abs(x[b, ~mask]) ** 2))
        on.append(np.mean(np.abs(x[b, mask]) ** 2))
    assert abs(np.mean(off) - 0.1) < 0.005
    assert abs(np.mean(on) - 1.1) < 0.02
    x2, _ = workloads.chirp_noise(n, batch=64)
    assert np.array_equal(x, x2)


def test_spectral_inputs():
    x, w = workloads.spectral_energy_inputs()
    assert x.shape == (512, 4096) and w.shape == (4096,) and w.dtype == np.float32
    assert np.all((w >= 0) & (w < 1))


def test_ragged_recipe():
    sizes, offs, data = workloads.ragged()
    assert sizes.shape == (2000,) and offs.shape == (2000,)
    assert set(np.unique(sizes)) <= set(workloads.SIZES)
    assert len(np.unique(sizes)) == 7
    assert offs[0] == 0 and np.all(np.diff(offs) == sizes[:-1])
    assert data.shape == (int(sizes.sum()),) and data.dtype == np.complex64
    # log-uniform exponents: each class near 2000/7
    counts = np.array([np.sum(sizes == s) for s in workloads.SIZES])
    assert np.all(np.abs(counts - 2000 / 7) < 60)


def test_bf16_rounding_is_nearest_even():
    # halfway cases round to the even neighbour; others to the nearest
    one = np.float32(1.0)
    step = np.float32(2.0 ** -7)  # bfloat16 spacing at 1.0
    vals = np.array([one, one + step / 2, one + 3 * step / 2, one + step / 4, -(one + step / 2),
                     np.float32(np.inf), np.float32(-0.0)], dtype=np.float32)
    got = workloads.bf16_value(workloads.bf16_bits(vals))
    want = np.array([1.0, 1.0, 1.0 + 2 * step, 1.0, -1.0, np.inf, -0.0], dtype=np.float32)
    assert np.array_equal(got, want)
    assert np.isnan(workloads.bf16_value(workloads.bf16_bits(np.array([np.nan], np.float32))))[0]


def test_storage_gate():
    x = workloads.plain_normal(256, 4, seed=3)
    for fmt, u in (("f16", 2.0 ** -11), ("bf16", 2.0 ** -8)):
        stored, v = workloads.to_storage(x, fmt)
        assert stored.shape == x.shape + (2,)
        ref = np.fft.fft(v)
        # the reference rounded once to the format passes ...
        _, r = workloads.to_storage(ref.astype(np.complex64), fmt)
        ok, worst, _, _ = metrics.gate_storage(r, ref, v, fmt)
        assert ok and worst <= u
        # ... ten roundings' worth of error does not
        bad = ref * (1 + 10 * u)
        assert not metrics.gate_storage(bad, ref, v, fmt)[0]


def test_dft16_real_matrix_form():
    # The 32 x 32 real form [[C, S], [-S, C]] acting on (Re x, Im x) is the
    # 16-point forward DFT (checked against numpy's FFT, an independent
    # routine); M / 4 is orthogonal, which is what lets one pass's relative
    # error be ||M_fmt - M||_2 / 4.
    k = np.arange(16)
    ang = 2.0 * np.pi * np.outer(k, k) / 16.0
    m = np.block([[np.cos(ang), np.sin(ang)], [-np.sin(ang), np.cos(ang)]])
    x = np.random.default_rng(4).standard_normal(16) + 1j * np.random.default_rng(5).standard_normal(16)
    y = m @ np.concatenate([x.real, x.imag])
    assert np.allclose(y[:16] + 1j * y[16:], np.fft.fft(x), rtol=0, atol=1e-12)
    assert np.allclose((m / 4) @ (m / 4).T, np.eye(32), atol=1e-14)


def test_mma_gate_factor():
    for fmt in ("f16", "bf16"):
        u = metrics.STORAGE_UNIT_ROUNDOFF[fmt]
        e = metrics.dft16_matrix_error(fmt)
        # the rounded matrix is off by less than one unit roundoff per pass, not 0
        assert 0 < e < u
        g = metrics.mma_gate_factor(fmt)
        assert g == pytest.approx(np.sqrt(4 / 3) + 3 * e / u)
    # binary16: cos(pi / 8), cos(pi / 4), cos(3 pi / 8) round by 5.6e-5, 1.1e-4
    # and 3.0e-4 relative, giving 0.258 u per pass
    assert metrics.dft16_matrix_error("f16") / 2.0 ** -11 == pytest.approx(0.2581, abs=1e-3)
    # pass counts: radix-16 passes on the matrix cores, then one smaller radix
    assert [metrics.mma_passes(n) for n in (512, 1024, 2048, 4096, 8192, 16384)] == \
        [(2, 3), (2, 3), (2, 3), (3, 3), (3, 4), (3, 4)]
    x = workloads.plain_normal(4096, 4, seed=3)
    stored, v = workloads.to_storage(x, "f16")
    ref = np.fft.fft(v)
    u = 2.0 ** -11
    g = metrics.mma_gate_factor("f16")
    # a relative error of 0.9 g u (every bin scaled) passes the matrix-core gate
    # and fails the single-rounding one; 1.1 g u fails both
    assert metrics.gate_storage(ref * (1 + 0.9 * g * u), ref, v, "f16", mma=True)[0]
    assert not metrics.gate_storage(ref * (1 + 0.9 * g * u), ref, v, "f16")[0]
    assert not metrics.gate_storage(ref * (1 + 1.1 * g * u), ref, v, "f16", mma=True)[0]
