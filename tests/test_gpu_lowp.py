"""16-bit storage (binary16 / bfloat16 pairs in HBM, FP32 arithmetic)
against the FP64 oracle applied to the stored input values."""
import ctypes

import numpy as np
import pytest

import oracle
import paper_2603_27569_amd as sf
from paper_2603_27569_amd import metrics, workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
DEV = "cuda:0"
SINGLE = [v for v in sf.variants() if v["kind"] == "single"]


def _device(stored, fmt):
    t = torch.from_numpy(np.ascontiguousarray(stored))
    if fmt == "bf16":
        t = t.view(torch.int16).view(torch.bfloat16)
    return t.to(DEV)


def _host(t, fmt):
    a = t.cpu()
    if fmt == "bf16":
        v = workloads.bf16_value(a.view(torch.int16).numpy().view(np.uint16)).astype(np.float64)
    else:
        v = a.numpy().astype(np.float64)
    return v[..., 0] + 1j * v[..., 1]


@pytest.mark.parametrize("fmt", ["f16", "bf16"])
@pytest.mark.parametrize("v", SINGLE, ids=[v["name"] for v in SINGLE])
def test_every_variant_with_16bit_storage(v, fmt):
    n = v["n"]
    batch = 2 * v["transforms_per_workgroup"] + 1
    x = workloads.plain_normal(n, batch, seed=n + 77)
    stored, xv = workloads.to_storage(x, fmt)
    for inverse in (False, True):
        p = sf.Plan(n, batch, sf.FFT_BACKWARD if inverse else sf.FFT_FORWARD,
                    sf.FFT_ALGO_SINGLE_PASS, v["name"])
        xt = _device(stored, fmt)
        yt = torch.empty_like(xt)
        sf.fft_exec_io(p.handle, xt.data_ptr(), yt.data_ptr(),
                       sf.FFT_IO_C16 if fmt == "f16" else sf.FFT_IO_BC16,
                       torch.cuda.current_stream().cuda_stream)
        torch.cuda.synchronize()
        p.close()
        ok, worst, _, ab = metrics.gate_storage(_host(yt, fmt), oracle.fft(xv, inverse=inverse), xv, fmt)
        assert ok, (inverse, worst, ab)


STREAMED = [v for v in SINGLE if v["streamed"]]


@pytest.mark.parametrize("fmt", ["f16", "bf16"])
@pytest.mark.parametrize("v", STREAMED, ids=[v["name"] for v in STREAMED])
def test_streamed_16bit_many_rows_per_workgroup(v, fmt):
    """16-bit storage through a persistent shape: several rows per
    workgroup, a ragged last round, both directions."""
    n = v["n"]
    g = torch.cuda.get_device_properties(0).multi_processor_count * v["streamed"]
    batch = 2 * g + 21
    x = workloads.plain_normal(n, batch, seed=n + 91)
    stored, xv = workloads.to_storage(x, fmt)
    for inverse in (False, True):
        p = sf.Plan(n, batch, sf.FFT_BACKWARD if inverse else sf.FFT_FORWARD,
                    sf.FFT_ALGO_SINGLE_PASS, v["name"])
        xt = _device(stored, fmt)
        yt = torch.empty_like(xt)
        sf.fft_exec_io(p.handle, xt.data_ptr(), yt.data_ptr(),
                       sf.FFT_IO_C16 if fmt == "f16" else sf.FFT_IO_BC16,
                       torch.cuda.current_stream().cuda_stream)
        torch.cuda.synchronize()
        p.close()
        ok, worst, _, ab = metrics.gate_storage(_host(yt, fmt), oracle.fft(xv, inverse=inverse), xv, fmt)
        assert ok, (inverse, worst, ab)


@pytest.mark.parametrize("fmt", ["f16", "bf16"])
def test_lowp_auto_plan_in_place_and_repeatable(fmt):
    n, b = 4096, 64
    x = workloads.plain_normal(n, b, seed=5)
    stored, xv = workloads.to_storage(x, fmt)
    xt = _device(stored, fmt)
    y1 = sf.fft_lowp(xt)
    y2 = sf.fft_lowp(xt)
    z = xt.clone()
    sf.fft_lowp(z, out=z)
    torch.cuda.synchronize()
    assert torch.equal(y1, y2) and torch.equal(y1, z)
    ok, worst, med, _ = metrics.gate_storage(_host(y1, fmt), oracle.fft(xv), xv, fmt)
    u = metrics.STORAGE_UNIT_ROUNDOFF[fmt]
    assert ok and med > 0.2 * u  # the error is the output rounding, not zero
    print(f"lowp {fmt}: worst rel-RMS {worst:.3e} (u = {u:.3e})", flush=True)


@pytest.mark.parametrize("fmt", ["f16", "bf16"])
@pytest.mark.parametrize("batch", [256, 2048, 16384])
def test_lowp_tuned_plans_at_bench_sizes_sampled_rows(fmt, batch):
    """The tuned 16-bit shapes at the batches the bench times (4096 x 256,
    2048, 16384; a persistent shape at 16384), both directions: rows sampled
    across the batch against the oracle on the stored values."""
    n = 4096
    g = torch.Generator(device=DEV)
    g.manual_seed(batch + 3)
    dt = torch.float16 if fmt == "f16" else torch.bfloat16
    xt = (torch.randn(batch, n, 2, device=DEV, generator=g)).to(dt)
    rows = sorted({0, 1, batch // 3, batch // 2 + 7, batch - 2, batch - 1})
    xv = _host(xt[rows], fmt)
    for inverse in (False, True):
        y = sf.fft_lowp(xt, inverse=inverse)
        ok, worst, _, ab = metrics.gate_storage(_host(y[rows], fmt), oracle.fft(xv, inverse=inverse),
                                                xv, fmt)
        assert ok, (inverse, worst, ab)
        del y
    del xt
    torch.cuda.empty_cache()


@pytest.mark.parametrize("fmt", ["f16", "bf16"])
def test_lowp_output_is_the_fp32_result_rounded_once(fmt):
    # The same plan in FP32 on the widened input gives the values before the
    # final rounding; the 16-bit result must be those, rounded to nearest
    # (within one unit in the last place where the two kernels' FP32
    # arithmetic differs in its last bit).
    n, b = 1024, 32
    x = workloads.plain_normal(n, b, seed=11)
    stored, xv = workloads.to_storage(x, fmt)
    xt = _device(stored, fmt)
    y16 = _host(sf.fft_lowp(xt), fmt)
    y32 = sf.fft(torch.from_numpy(xv.astype(np.complex64)).to(DEV), algorithm=sf.FFT_ALGO_SINGLE_PASS)
    _, r32 = workloads.to_storage(y32.cpu().numpy(), fmt)
    torch.cuda.synchronize()
    same = np.mean(y16 == r32)
    assert same > 0.99, same
    u = metrics.STORAGE_UNIT_ROUNDOFF[fmt]
    rowmax = np.max(np.abs(r32), axis=1, keepdims=True)
    assert np.all(np.abs(y16 - r32) <= 4 * u * (np.abs(r32) + 1e-3 * rowmax))


def test_lowp_errors():
    L = sf._lib.lib()
    vp = ctypes.c_void_p
    buf = torch.zeros(4096 * 8, dtype=torch.float16, device=DEV)
    base = buf.data_ptr()
    p = sf.Plan(1024, 4)
    assert L.fft_exec_io(vp(p.handle), vp(base + 2), vp(base + 8192), 1, None) == sf.CODES["FFT_MISALIGNED"]
    assert L.fft_exec_io(vp(p.handle), vp(base), vp(base + 4), 1, None) == sf.CODES["FFT_OVERLAP"]
    assert L.fft_exec_io(vp(p.handle), vp(base), vp(base), 7, None) == sf.CODES["FFT_INVALID_ARGUMENT"]
    q = sf.Plan(8192, 1, algorithm=sf.FFT_ALGO_FOUR_STEP)
    assert L.fft_exec_io(vp(q.handle), vp(base), vp(base), 2, None) == sf.CODES["FFT_UNSUPPORTED"]
    q.close()
    h = p.handle
    p.close()
    assert L.fft_exec_io(vp(h), vp(base), vp(base), 1, None) == sf.CODES["FFT_INVALID_PLAN"]
    torch.cuda.synchronize()


# ---------------------------------------------------------------- matrix cores
# FFT_IO_C16_MMA / FFT_IO_BC16_MMA: N = 16^P RL from 512 to 16384, the 16-point
# DFTs of the radix-16 passes as matrix-core products with 16-bit operands and
# FP32 sums (then one radix-RL pass on the vector ALUs), gated by
# metrics.gate_storage(..., mma=True).

MMA_SIZES = [512, 1024, 2048, 4096, 8192, 16384]

MMA_IO = {"f16": sf.FFT_IO_C16_MMA, "bf16": sf.FFT_IO_BC16_MMA}


def _run_io(plan, xt, io, out=None):
    yt = torch.empty_like(xt) if out is None else out
    sf.fft_exec_io(plan.handle, xt.data_ptr(), yt.data_ptr(), io,
                   torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    return yt


@pytest.mark.parametrize("fmt", ["f16", "bf16"])
@pytest.mark.parametrize("inverse", [False, True], ids=["forward", "backward"])
@pytest.mark.parametrize("n,batch", [(4096, 1), (4096, 9)] + [(m, 5) for m in MMA_SIZES if m != 4096])
def test_mma_matches_oracle(fmt, inverse, n, batch):
    x = workloads.plain_normal(n, batch, seed=40 + batch + n)
    stored, xv = workloads.to_storage(x, fmt)
    p = sf.Plan(n, batch, sf.FFT_BACKWARD if inverse else sf.FFT_FORWARD, sf.FFT_ALGO_SINGLE_PASS)
    y = _host(_run_io(p, _device(stored, fmt), MMA_IO[fmt]), fmt)
    p.close()
    ok, worst, med, ab = metrics.gate_storage(y, oracle.fft(xv, inverse=inverse), xv, fmt, mma=True)
    u = metrics.STORAGE_UNIT_ROUNDOFF[fmt]
    p16, ptot = metrics.mma_passes(n)
    print(f"mma {fmt} n={n} inverse={inverse} b={batch}: worst rel-RMS {worst / u:.3f} u, "
          f"gate {metrics.mma_gate_factor(fmt, ptot, p16):.3f} u, bin ratio {ab:.3f}", flush=True)
    assert ok, (worst / u, ab)
    assert med > 0.2 * u  # the path rounds; an exact result would mean it did not run


@pytest.mark.parametrize("fmt", ["f16", "bf16"])
@pytest.mark.parametrize("n", [1024, 4096])
def test_mma_any_plan_variant_and_closed_forms(fmt, n):
    # The kernel runs on the plan's twiddle table when the plan's variant has
    # its radix plan, else on a table of its own: every variant's plan gives
    # the same answer.  Closed forms: a delta row gives all ones, a tone
    # e^{2 pi i k0 n / N} gives N at bin k0 (within the gate).
    rows = np.zeros((3, n), dtype=np.complex128)
    rows[0, 0] = 1.0
    rows[1] = np.exp(2j * np.pi * 37 * np.arange(n) / n) / 64.0  # N / 64 at bin 37
    rows[2] = workloads.plain_normal(n, 1, seed=2)[0]
    stored, xv = workloads.to_storage(rows, fmt)
    ref = oracle.fft(xv)
    for v in SINGLE:
        if v["n"] != n:
            continue
        p = sf.Plan(n, 3, sf.FFT_FORWARD, sf.FFT_ALGO_SINGLE_PASS, v["name"])
        y = _host(_run_io(p, _device(stored, fmt), MMA_IO[fmt]), fmt)
        p.close()
        ok, worst, _, ab = metrics.gate_storage(y, ref, xv, fmt, mma=True)
        assert ok, (v["name"], worst, ab)
        assert np.all(y[0] == 1.0), v["name"]  # pass 0 of a delta is exact, later passes see ones


def test_mma_large_batch_split_in_place_and_repeatable():
    n, b = 4096, 20000
    gen = np.random.default_rng(8)
    xt = torch.from_numpy(gen.standard_normal((b, n, 2)).astype(np.float16)).to(DEV)
    p = sf.Plan(n, b, sf.FFT_FORWARD, sf.FFT_ALGO_SINGLE_PASS)
    y1 = _run_io(p, xt, sf.FFT_IO_C16_MMA)
    y2 = _run_io(p, xt, sf.FFT_IO_C16_MMA)
    try:
        sf.fft_set_launch_limit(4097)  # several grids per call
        y3 = _run_io(p, xt, sf.FFT_IO_C16_MMA)
    finally:
        sf.fft_set_launch_limit(0)
    z = xt.clone()
    _run_io(p, z, sf.FFT_IO_C16_MMA, out=z)
    yv = _run_io(p, xt, sf.FFT_IO_C16)
    p.close()
    assert torch.equal(y1, y2) and torch.equal(y1, y3) and torch.equal(y1, z)
    assert not torch.equal(y1, yv)  # a different kernel from the FP32-arithmetic one
    rows = [0, 1, 4095, 4096, 12345, b - 1]
    xs = xt[rows].cpu().numpy().astype(np.float64)
    xv = xs[..., 0] + 1j * xs[..., 1]
    ok, worst, _, ab = metrics.gate_storage(_host(y1[rows], "f16"), oracle.fft(xv), xv, "f16", mma=True)
    assert ok, (worst, ab)


@pytest.mark.parametrize("fmt", ["f16", "bf16"])
@pytest.mark.parametrize("batch", [700, 5000], ids=["two_waves", "one_wave"])
def test_mma_lanes_per_transform_by_batch(fmt, batch):
    # Larger batches run the kernel with two waves, then one wave, per
    # transform: sampled rows against the oracle, both directions.
    n = 4096
    x = workloads.plain_normal(n, batch, seed=batch)
    stored, xv = workloads.to_storage(x, fmt)
    rows = [0, 1, batch // 2, batch - 1]
    xt = _device(stored, fmt)
    for inverse in (False, True):
        p = sf.Plan(n, batch, sf.FFT_BACKWARD if inverse else sf.FFT_FORWARD,
                    sf.FFT_ALGO_SINGLE_PASS)
        y = _host(_run_io(p, xt, MMA_IO[fmt])[rows], fmt)
        p.close()
        ok, worst, _, ab = metrics.gate_storage(y, oracle.fft(xv[rows], inverse=inverse), xv[rows],
                                                fmt, mma=True)
        assert ok, (inverse, worst, ab)


def test_mma_unsupported_plans():
    L = sf._lib.lib()
    vp = ctypes.c_void_p
    buf = torch.zeros(65536 * 4, dtype=torch.float16, device=DEV)
    base = buf.data_ptr()
    for args in ((256, 2, sf.FFT_FORWARD, sf.FFT_ALGO_SINGLE_PASS),
                 (8192, 1, sf.FFT_FORWARD, sf.FFT_ALGO_FOUR_STEP),
                 (65536, 1, sf.FFT_FORWARD)):
        p = sf.Plan(*args)
        for io in (sf.FFT_IO_C16_MMA, sf.FFT_IO_BC16_MMA):
            assert L.fft_exec_io(vp(p.handle), vp(base), vp(base), io, None) == \
                sf.CODES["FFT_UNSUPPORTED"], args
        p.close()
    torch.cuda.synchronize()
