"""GPU parity of the HIP path against the FP64 oracle.

Every case runs the library through its C ABI (via the Python binding) on
seeded inputs and compares element by element with the oracle on the same
complex64 values.  Gates (per row, worst row decides): relative RMS error
<= 5e-6 and max abs error <= 1e-5 * ||x_b||_2.
"""
import numpy as np
import pytest

import oracle
import paper_2603_27569_amd as sf
from paper_2603_27569_amd import metrics, workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _gpu(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to(DEV)


def _host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _check(y, x, inverse=False, ref=None):
    if ref is None:
        ref = oracle.fft(x, inverse=inverse)
    ok, worst, med, ab = metrics.gate(y, ref, x)
    assert ok, f"rel-RMS worst {worst:.3e} median {med:.3e} max-abs/||x|| {ab:.3e}"
    return worst


SINGLE = [v for v in sf.variants() if v["kind"] == "single"]
FOUR = [v for v in sf.variants() if v["kind"] == "four_step"]


@pytest.mark.parametrize("v", SINGLE, ids=[v["name"] for v in SINGLE])
@pytest.mark.parametrize("inverse", [False, True], ids=["fwd", "bwd"])
def test_single_pass_variant_parity(v, inverse):
    n = v["n"]
    batch = 3 * v["transforms_per_workgroup"] + 1  # a ragged last workgroup
    x = workloads.plain_uniform(n, batch, seed=n + batch)
    y = sf.fft(_gpu(x), inverse=inverse, algorithm=sf.FFT_ALGO_SINGLE_PASS, variant=v["name"])
    worst = _check(_host(y), x, inverse)
    assert worst < 2e-6  # a healthy FP32 Stockham sits near 1e-7


WAVEX = [v for v in SINGLE if v["wave_exchange"]]


@pytest.mark.parametrize("v", WAVEX, ids=[v["name"] for v in WAVEX])
def test_in_wave_exchange_in_place_round_trip(v):
    """The in-wave shapes in place (out == in): every lane has consumed its row
    before the workgroup's one barrier and stores after it.  Forward, then
    backward, both in place, and the result against the oracle at each step."""
    n, batch = v["n"], 37
    x = workloads.plain_normal(n, batch, seed=900 + v["values_per_lane"])
    xt = _gpu(x)
    sf.fft(xt, out=xt, algorithm=sf.FFT_ALGO_SINGLE_PASS, variant=v["name"])
    y = _host(xt)
    _check(y, x)
    sf.fft(xt, inverse=True, out=xt, algorithm=sf.FFT_ALGO_SINGLE_PASS, variant=v["name"])
    _check(_host(xt), y, inverse=True)


STREAMED = [v for v in SINGLE if v["streamed"]]


@pytest.mark.parametrize("v", STREAMED, ids=[v["name"] for v in STREAMED])
@pytest.mark.parametrize("inverse", [False, True], ids=["fwd", "bwd"])
def test_streamed_variant_many_rows_per_workgroup(v, inverse):
    """A persistent shape's workgroups loop over the rows (row = id + i G with
    G = streamed x CUs): two full rounds and a ragged third, out of place and
    in place (a row is read before it is written, and the prefetched row is
    another one)."""
    n = v["n"]
    g = torch.cuda.get_device_properties(0).multi_processor_count * v["streamed"]
    batch = 2 * g + 37
    x = workloads.plain_uniform(n, batch, seed=n + batch + 11)
    ref = oracle.fft(x, inverse=inverse)
    y = sf.fft(_gpu(x), inverse=inverse, algorithm=sf.FFT_ALGO_SINGLE_PASS, variant=v["name"])
    assert _check(_host(y), x, inverse, ref=ref) < 2e-6
    xt = _gpu(x)
    sf.fft(xt, inverse=inverse, out=xt, algorithm=sf.FFT_ALGO_SINGLE_PASS, variant=v["name"])
    assert _check(_host(xt), x, inverse, ref=ref) < 2e-6
    assert v["fused_kernel"] and not v["fused_kernels"]  # no matched filter


@pytest.mark.parametrize("v", FOUR, ids=[v["name"] for v in FOUR])
@pytest.mark.parametrize("inverse", [False, True], ids=["fwd", "bwd"])
def test_four_step_variant_parity(v, inverse):
    n = v["n"]
    batch = 13  # not a multiple of the 8-row XCD group
    x = workloads.plain_normal(n, batch, seed=n + 7)
    y = sf.fft(_gpu(x), inverse=inverse, algorithm=sf.FFT_ALGO_FOUR_STEP, variant=v["name"])
    _check(_host(y), x, inverse)


@pytest.mark.parametrize("n", [1 << 15, 1 << 17, 1 << 20])
def test_large_n_auto_plan_closed_forms(n):
    # Beyond 16384 the default plan is the four-step; a shifted delta gives
    # W_N^{n0 k} and a tone gives one bin of height N.
    n0, k0 = 12345 % n, (77 * n) // 100 + 3
    x = np.zeros((2, n), np.complex64)
    x[0, n0] = 1.0
    m = np.arange(n)
    x[1] = np.exp(2j * np.pi * ((k0 * m) % n) / n).astype(np.complex64)
    y = _host(sf.fft(_gpu(x)))
    _check(y, x)
    exact = np.exp(-2j * np.pi * ((n0 * m) % n) / n)
    assert np.max(np.abs(y[0] - exact)) <= 1e-5
    assert int(np.argmax(np.abs(y[1]))) == k0
    assert abs(y[1, k0] - n) <= 1e-5 * n
    p = sf.Plan(n, 2)
    assert p.describe()["algorithm"] == "four_step"
    p.close()
    with pytest.raises(sf.StockfftError) as e:
        sf.Plan(n, 2, algorithm=sf.FFT_ALGO_SINGLE_PASS)
    assert e.value.name == "FFT_UNSUPPORTED"


@pytest.mark.parametrize("n", list(workloads.SIZES) + [1 << 15])
def test_single_row_auto_plan(n):
    # batch 1: the tuned choice for the smallest bucket (a four-step split at
    # 8192 and 16384, fewer workgroups than CUs everywhere)
    x = workloads.plain_normal(n, 1, seed=n + 3)
    _check(_host(sf.fft(_gpu(x))), x)
    _check(_host(sf.fft(_gpu(x), inverse=True)), x, inverse=True)


@pytest.mark.parametrize("n,batch", [(16384, 8192), (256, 1 << 20), (4096, 16384)])
def test_large_batch_sampled_rows(n, batch):
    # A 1-2 GiB batch generated on the device; rows sampled across it (first,
    # last, and strided) are checked against the oracle one by one.  At
    # 4096 x 16384 the tuned plan is a persistent shape (rows looped over by
    # a few workgroups per CU), checked in both directions.
    g = torch.Generator(device=DEV)
    g.manual_seed(n + batch)
    x = torch.randn(batch, n, dtype=torch.complex64, device=DEV, generator=g)
    rows = sorted({0, 1, batch // 3, batch // 2 + 7, batch - 2, batch - 1})
    xs = _host(x[rows])
    for inverse in ((False, True) if n == 4096 else (False,)):
        y = sf.fft(x, inverse=inverse)
        _check(_host(y[rows]), xs, inverse)
        del y
    del x
    torch.cuda.empty_cache()


def test_plain_uniform_n256_delta_tone():
    n, b = 256, 64
    x = workloads.plain_uniform(n, b)
    _check(_host(sf.fft(_gpu(x))), x)
    d = workloads.delta_batch(n, b)
    y = _host(sf.fft(_gpu(d)))
    k = np.arange(n)
    for r in range(b):
        n0 = r % n
        exact = np.exp(-2j * np.pi * ((n0 * k) % n) / n)
        assert np.max(np.abs(y[r] - exact)) < 2e-6
    t = workloads.tone_batch(n, b)
    y = _host(sf.fft(_gpu(t)))
    bins = workloads.tone_bins(n, b)
    for r in range(b):
        z = y[r].copy()
        assert abs(z[bins[r]] - n) < 1e-3
        z[bins[r]] = 0
        assert np.max(np.abs(z)) < 1e-3
    _check(y, t)


@pytest.mark.parametrize("inverse", [False, True], ids=["fwd", "bwd"])
def test_headline_n4096_b256(inverse):
    x = workloads.plain_normal(4096, 256)
    y = _host(sf.fft(_gpu(x), inverse=inverse))
    worst = _check(y, x, inverse)
    print(f"n4096 b256 inverse={inverse} worst rel-RMS {worst:.3e}", flush=True)


@pytest.mark.parametrize("n", [8192, 16384])
@pytest.mark.parametrize("algo", [sf.FFT_ALGO_SINGLE_PASS, sf.FFT_ALGO_FOUR_STEP], ids=["single", "fourstep"])
def test_chirp_noise_b1024(n, algo):
    x, _ = workloads.chirp_noise(n, 1024)
    y = _host(sf.fft(_gpu(x), algorithm=algo))
    worst = _check(y, x)
    print(f"chirp n{n} algo={algo} worst rel-RMS {worst:.3e}", flush=True)


@pytest.mark.parametrize("n", workloads.SIZES)
def test_roundtrip_in_place_and_determinism(n):
    x = workloads.plain_normal(n, 5, seed=3)
    xt = _gpu(x)
    y1 = sf.fft(xt)
    y2 = sf.fft(xt)
    assert torch.equal(y1, y2)  # bitwise run to run
    back = _host(sf.fft(y1, inverse=True)) / n
    assert np.max(np.abs(back - x)) < 1e-5 * np.max(np.abs(x)) * np.log2(n)
    z = xt.clone()
    sf.fft(z, out=z)  # in place
    assert torch.equal(z, y1)


@pytest.mark.parametrize("algo", [sf.FFT_ALGO_SINGLE_PASS, sf.FFT_ALGO_FOUR_STEP])
def test_zero_rows_are_exact_zeros(algo):
    x = np.zeros((9, 8192), np.complex64)
    x[3] = workloads.plain_normal(8192, 1)[0]
    y = _host(sf.fft(_gpu(x), algorithm=algo))
    assert np.all(y[[0, 1, 2, 4, 5, 6, 7, 8]] == 0)
    _check(y, x)


def test_exec_pointer_errors():
    n, b = 1024, 4
    p = sf.Plan(n, b)
    buf = torch.zeros(2 * n * b + 8, dtype=torch.complex64, device=DEV)
    base = buf.data_ptr()
    codes = sf.CODES
    L = sf._lib.lib()
    import ctypes
    vp = ctypes.c_void_p
    assert L.fft_exec(vp(p.handle), vp(base + 4), vp(base + 16 * n * b), None) == codes["FFT_MISALIGNED"]
    assert L.fft_exec(vp(p.handle), vp(base), vp(base + 8), None) == codes["FFT_OVERLAP"]
    assert L.fft_exec(vp(p.handle), None, vp(base), None) == codes["FFT_INVALID_POINTER"]
    assert L.fft_exec(vp(p.handle), vp(base), vp(base + 8 * n * b), None) == 0  # adjacent is fine
    h = p.handle
    p.close()
    assert L.fft_exec(vp(h), vp(base), vp(base), None) == codes["FFT_INVALID_PLAN"]
    assert L.fft_destroy(vp(h)) == codes["FFT_INVALID_PLAN"]
    torch.cuda.synchronize()


def test_plan_describe_and_alloc_failure(monkeypatch):
    p = sf.Plan(16384, 3, algorithm=sf.FFT_ALGO_FOUR_STEP)
    d = p.describe()
    assert d["algorithm"] == "four_step" and d["workspace_bytes"] == 16384 * 3 * 8
    assert d["four_step"]["n1"] * d["four_step"]["n2"] == 16384
    p.close()
    # the compiled kernel's resources as the runtime reports them (the
    # headline shape: no scratch, its static LDS as the variant states)
    p = sf.Plan(4096, 256, variant="n4096_e8_b1_p4_r8.8.8.8_pt")
    r = p.describe()["variant_resources"]
    assert 0 < r["vgprs"] <= 128 and r["scratch_bytes_per_lane"] == 0
    assert r["lds_bytes"] == p.describe()["variant"]["lds_bytes"] and r["max_threads"] >= 512
    p.close()
    monkeypatch.setenv("STOCKFFT_FAIL_ALLOC", "1")
    with pytest.raises(sf.StockfftError) as e:
        sf.Plan(4096, 3)
    assert e.value.name == "FFT_ALLOC_FAILED"


def test_launch_splitting_matches_single_grid():
    try:
        sf.fft_set_launch_limit(3)
        # (the tiled splits at 2^17 and 2^20: one row per launch, grids rounded
        # up to whole XCD groups)
        for n, algo, b in [(256, sf.FFT_ALGO_SINGLE_PASS, 200), (8192, sf.FFT_ALGO_FOUR_STEP, 21),
                           (1 << 17, sf.FFT_ALGO_FOUR_STEP, 3), (1 << 20, sf.FFT_ALGO_FOUR_STEP, 2)]:
            x = workloads.plain_normal(n, b, seed=5)
            sf.clear_plan_cache()
            y = _host(sf.fft(_gpu(x), algorithm=algo))
            _check(y, x)
    finally:
        sf.fft_set_launch_limit(0)
        sf.clear_plan_cache()


# ------------------------------------------------------------- fused paths

def test_spectral_energy_fused_matches_oracle():
    x, w = workloads.spectral_energy_inputs()
    xt, wt = _gpu(x), _gpu(w)
    total, rows, grad = sf.spectral_energy(xt, wt)
    rows = _host(rows).astype(np.float64)
    grad = _host(grad)
    ref_rows, ref_grad = oracle.spectral_energy(x, w)
    assert np.max(np.abs(rows - ref_rows) / ref_rows) <= 1e-5
    assert abs(float(_host(total)[0]) - ref_rows.sum()) / ref_rows.sum() <= 1e-5
    ok, worst, ab = metrics.grad_gate(grad, ref_grad)
    assert ok, f"worst row grad rel {worst:.3e}, max-abs/||g_ref|| {ab:.3e}"
    print(f"spectral energy worst row grad rel {worst:.3e}", flush=True)
    # Central differences on the FP64 oracle (exact: the loss is quadratic).
    g = np.random.default_rng(0)
    for _ in range(6):
        b, i = int(g.integers(512)), int(g.integers(4096))
        for comp in (1.0, 1j):
            e = np.zeros((1, 4096), complex)
            e[0, i] = comp
            lp = oracle.spectral_energy(x[b:b + 1] + e, w)[0].sum()
            lm = oracle.spectral_energy(x[b:b + 1] - e, w)[0].sum()
            fd = (lp - lm) / 2.0
            got = grad[b, i].real if comp == 1.0 else grad[b, i].imag
            assert abs(got - fd) <= 1e-4 * np.max(np.abs(ref_grad[b])), (b, i, comp)


@pytest.mark.parametrize("n,batch", [(1024, 2000), (4096, 256), (4096, 512), (4096, 1200), (16384, 600)])
def test_spectral_energy_takes_its_own_tuned_shape(n, batch):
    # The fused kernel runs two transforms per load and has a tuned table of
    # its own (here a choice that differs from the plain transform's); its
    # results still match the oracle.
    p = sf.Plan(n, batch, sf.FFT_FORWARD, sf.FFT_ALGO_SINGLE_PASS)
    d = p.describe()
    p.close()
    assert d["fused_variant"] == sf.fft_tune_query_fused(n, batch)
    assert d["filter_variant"] == sf.fft_tune_query_filter(n, batch)
    assert d["fused_variant"] != d["variant"]["name"]
    x, w = workloads.spectral_energy_inputs(n=n, batch=batch, seed=41, wseed=42)
    total, rows, grad = sf.spectral_energy(_gpu(x), _gpu(w))
    ref_rows, ref_grad = oracle.spectral_energy(x, w)
    rows = _host(rows).astype(np.float64)
    assert np.max(np.abs(rows - ref_rows) / ref_rows) <= 1e-5
    assert abs(float(_host(total)[0]) - ref_rows.sum()) / ref_rows.sum() <= 1e-5
    ok, worst, ab = metrics.grad_gate(_host(grad), ref_grad)
    assert ok, (worst, ab)


FUSED = [v for v in SINGLE if v["fused_kernel"]]


@pytest.mark.parametrize("v", FUSED, ids=[v["name"] for v in FUSED])
def test_spectral_energy_every_fused_variant(v):
    """Every shape with the fused forward -> weight -> adjoint kernel, named
    explicitly: per-row loss, per-row gradient gate and the fixed-order loss
    total against the oracle.  Persistent shapes get two full rounds of rows
    and a ragged third (each workgroup loops and prefetches)."""
    n = v["n"]
    if v["streamed"]:
        batch = 2 * torch.cuda.get_device_properties(0).multi_processor_count * v["streamed"] + 37
    else:
        batch = 3 * v["transforms_per_workgroup"] + 1
    x, w = workloads.spectral_energy_inputs(n=n, batch=batch, seed=n + batch, wseed=n + 1)
    xt, wt = _gpu(x), _gpu(w)
    p = sf.Plan(n, batch, sf.FFT_FORWARD, sf.FFT_ALGO_SINGLE_PASS, v["name"])
    assert p.describe()["fused_variant"] == v["name"]
    rows = torch.empty(batch, device=DEV)
    total = torch.empty(1, device=DEV)
    grad = torch.empty_like(xt)
    cs = torch.cuda.current_stream().cuda_stream
    sf.fft_exec_spectral_energy(p.handle, xt.data_ptr(), wt.data_ptr(), 0, grad.data_ptr(),
                                rows.data_ptr(), total.data_ptr(), cs)
    torch.cuda.synchronize()
    p.close()
    ref_rows, ref_grad = oracle.spectral_energy(x, w)
    got_rows = _host(rows).astype(np.float64)
    assert np.max(np.abs(got_rows - ref_rows) / ref_rows) <= 1e-5
    assert float(_host(total)[0]) == _fixed_order_total(_host(rows))
    ok, worst, ab = metrics.grad_gate(_host(grad), ref_grad)
    assert ok, (worst, ab)


def test_spectral_energy_loss_only_and_scale():
    x, w = workloads.spectral_energy_inputs(n=1024, batch=40)
    xt, wt = _gpu(x), _gpu(w)
    t1, r1, g1 = sf.spectral_energy(xt, wt, want_grad=False)
    assert g1 is None
    t2, r2, g2 = sf.spectral_energy(xt, wt, grad_scale=torch.tensor([-0.5], device=DEV))
    assert torch.equal(r1, r2)
    _, ref = oracle.spectral_energy(x, w)
    ok, worst, ab = metrics.grad_gate(_host(g2), -0.5 * ref)
    assert ok, (worst, ab)


def _fixed_order_total(rows):
    """The loss total's summation order written out on the host in FP32:
    1024 lanes each add rows i, i + 1024, ...; then a halving tree (lane t
    adds lane t + w for w = 512, 256, ..., 1)."""
    r = np.asarray(rows, dtype=np.float32)
    lanes = np.zeros(1024, dtype=np.float32)
    for i in range(0, len(r), 1024):
        chunk = r[i:i + 1024]
        lanes[:len(chunk)] = lanes[:len(chunk)] + chunk
    w = 512
    while w > 0:
        lanes[:w] = lanes[:w] + lanes[w:2 * w]
        w //= 2
    return float(lanes[0])


@pytest.mark.parametrize("n,batch", [(2048, 3000), (4096, 300)], ids=["n2048", "n4096_in_wave"])
@pytest.mark.parametrize("limit", [0, 7], ids=["one_launch", "split_launches"])
def test_spectral_energy_total_reproducible(limit, n, batch):
    # The loss total must cover every row (also when the fused kernel is split
    # over several launches), equal the fixed-order sum of the row losses bit
    # for bit, and repeat exactly from call to call.  (At 4096 x 300 the tuned
    # shape is the in-wave kernel, which counts each workgroup before its
    # adjoint.)
    x, w = workloads.spectral_energy_inputs(n=n, batch=batch, seed=21, wseed=22)
    xt, wt = _gpu(x), _gpu(w)
    try:
        sf.fft_set_launch_limit(limit)
        sf.clear_plan_cache()
        totals = []
        for _ in range(3):
            total, rows, _ = sf.spectral_energy(xt, wt, want_grad=(len(totals) != 1))
            torch.cuda.synchronize()
            totals.append(float(_host(total)[0]))
    finally:
        sf.fft_set_launch_limit(0)
        sf.clear_plan_cache()
    assert totals[0] == totals[1] == totals[2]
    assert totals[0] == _fixed_order_total(_host(rows))
    ref_rows, _ = oracle.spectral_energy(x, w)
    assert abs(totals[0] - ref_rows.sum()) / ref_rows.sum() <= 1e-5


@pytest.mark.parametrize("n,batch", [(256, 5), (4096, 17), (16384, 40)])
def test_spectral_energy_total_few_workgroups(n, batch):
    # Fewer workgroups than the total's first-level counters, and several rows
    # per workgroup: the total still covers every row exactly once, in the
    # fixed order, on repeated calls (the counters must come back to zero).
    x, w = workloads.spectral_energy_inputs(n=n, batch=batch, seed=31, wseed=32)
    xt, wt = _gpu(x), _gpu(w)
    totals = []
    for want in (True, False, True):
        total, rows, _ = sf.spectral_energy(xt, wt, want_grad=want)
        totals.append(float(_host(total)[0]))
    assert totals[0] == totals[1] == totals[2]
    assert totals[0] == _fixed_order_total(_host(rows))
    ref_rows, _ = oracle.spectral_energy(x, w)
    assert abs(totals[0] - ref_rows.sum()) / ref_rows.sum() <= 1e-5


def test_spectral_energy_unit_weight_closed_form():
    n = 4096
    x = workloads.plain_normal(n, 8, seed=9)
    _, rows, grad = sf.spectral_energy(_gpu(x), torch.ones(n, device=DEV))
    grad = _host(grad)
    ok, worst, ab = metrics.grad_gate(grad, 2 * n * x.astype(np.complex128))
    assert ok and worst <= 1e-5, (worst, ab)
    rows = _host(rows)
    ref = n * np.sum(np.abs(x.astype(np.complex128)) ** 2, axis=1)
    assert np.max(np.abs(rows - ref) / ref) <= 1e-5


def test_autograd_functions():
    x, w = workloads.spectral_energy_inputs(n=2048, batch=16)
    _, ref = oracle.spectral_energy(x, w)
    xt = _gpu(x).requires_grad_(True)
    wt = _gpu(w)
    loss = sf.SpectralEnergyFunction.apply(xt, wt) * 3.0
    loss.backward()
    ok, worst, ab = metrics.grad_gate(_host(xt.grad), 3 * ref)
    assert ok, (worst, ab)
    # The same gradient through FFTFunction and plain torch elementwise ops.
    xt2 = _gpu(x).requires_grad_(True)
    y = sf.FFTFunction.apply(xt2)
    l2 = (wt ** 2 * (y.real ** 2 + y.imag ** 2)).sum()
    l2.backward()
    ok, worst, ab = metrics.grad_gate(_host(xt2.grad), ref)
    assert ok, (worst, ab)


@pytest.mark.parametrize("n", [1024, 4096, 16384])
def test_matched_filter_every_variant_and_tuned_choice(n):
    # The filter kernel is tuned separately from the plain transform: the
    # plan's own choice (with its own twiddle table) and every variant named
    # explicitly must all match the oracle.
    b = 9
    x = workloads.plain_normal(n, b, seed=n + 1)
    h = workloads.complex_normal((n,), seed=n + 2)
    ref = oracle.matched_filter(x, h)
    xt, ht = _gpu(x), _gpu(h)
    names = [None] + [v["name"] for v in SINGLE if v["n"] == n and v["fused_kernels"]]
    for name in names:
        p = sf.Plan(n, b, sf.FFT_FORWARD, sf.FFT_ALGO_SINGLE_PASS, name)
        d = p.describe()
        want = name if name else sf.fft_tune_query_filter(n, b)
        assert d["filter_variant"] == want
        y = torch.empty_like(xt)
        sf.fft_exec_matched_filter(p.handle, xt.data_ptr(), ht.data_ptr(), y.data_ptr(),
                                   torch.cuda.current_stream().cuda_stream)
        torch.cuda.synchronize()
        ok, worst, _, ab = metrics.gate(_host(y), ref, x)
        assert ok, (name, worst, ab)
        p.close()


def test_matched_filter_matches_oracle():
    n, b = 4096, 33
    x = workloads.plain_normal(n, b, seed=12)
    h = workloads.complex_normal((n,), seed=13)
    y = _host(sf.matched_filter(_gpu(x), _gpu(h)))
    ref = oracle.matched_filter(x, h)
    ok, worst, _, ab = metrics.gate(y, ref, x)
    assert ok, (worst, ab)


def test_two_streams_same_shape_four_step():
    # A four-step plan owns one workspace: the plan cache keys plans by
    # stream, so two streams transforming the same shape at once each get a
    # plan (and a workspace) of their own.
    n, b = 16384, 32
    xa = workloads.plain_normal(n, b, seed=61)
    xb = workloads.plain_normal(n, b, seed=62)
    ta, tb = _gpu(xa), _gpu(xb)
    sa, sb = torch.cuda.Stream(), torch.cuda.Stream()
    torch.cuda.synchronize()
    outs = []
    for _ in range(4):
        with torch.cuda.stream(sa):
            ya = sf.fft(ta, algorithm=sf.FFT_ALGO_FOUR_STEP)
        with torch.cuda.stream(sb):
            yb = sf.fft(tb, algorithm=sf.FFT_ALGO_FOUR_STEP)
        outs.append((ya, yb))
    torch.cuda.synchronize()
    pa = sf.cached_plan(n, b, sf.FFT_FORWARD, 0, sf.FFT_ALGO_FOUR_STEP, None, sa.cuda_stream)
    pb = sf.cached_plan(n, b, sf.FFT_FORWARD, 0, sf.FFT_ALGO_FOUR_STEP, None, sb.cuda_stream)
    assert pa is not pb and pa.describe()["algorithm"] == "four_step"
    ra, rb = oracle.fft(xa), oracle.fft(xb)
    for ya, yb in outs:
        _check(_host(ya), xa, ref=ra)
        _check(_host(yb), xb, ref=rb)
