"""The measurement references of libstockref.so on the GPU: the copies move
the bytes exactly, the two chain steps compute what the fused kernels fuse,
and the stamped transform gives the transform's result with ordered stamps."""
import numpy as np
import pytest

import oracle
import paper_2603_27569_amd as sf
from paper_2603_27569_amd import metrics, reference as ref, workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _cs():
    return torch.cuda.current_stream().cuda_stream


@pytest.mark.parametrize("n,lanes,batch", [(4096, 256, 37), (4096, 512, 3), (4096, 1024, 2),
                                           (1024, 64, 5), (16384, 1024, 2)])
def test_copy_rows_exact(n, lanes, batch):
    x = torch.randn(batch, n, dtype=torch.complex64, device=DEV)
    y = torch.zeros_like(x)
    ref.copy_rows(x.data_ptr(), y.data_ptr(), n, batch, lanes, _cs())
    torch.cuda.synchronize()
    assert torch.equal(x, y)


@pytest.mark.parametrize("groups,rounds", [(1, 0), (3, 1), (256, 7), (40, 300)])
def test_lds_exchange_moves_every_value(groups, rounds):
    out = torch.full((groups * 256,), -1.0, dtype=torch.float32, device=DEV)
    ref.lds_exchange(groups, rounds, out.data_ptr(), _cs())
    torch.cuda.synchronize()
    t = np.arange(256)
    want = np.tile(16 * ((t + rounds) % 256) + 120, groups).astype(np.float32)
    assert np.array_equal(out.cpu().numpy(), want)


@pytest.mark.parametrize("nbytes", [16, 4096 * 16, 4096 * 16 * 3 + 48])
def test_copy_wide_exact_and_bounded(nbytes):
    src = torch.randint(0, 255, (nbytes + 64,), dtype=torch.uint8, device=DEV)
    dst = torch.zeros(nbytes + 64, dtype=torch.uint8, device=DEV)
    ref.copy_wide(src.data_ptr(), dst.data_ptr(), nbytes, _cs())
    torch.cuda.synchronize()
    assert torch.equal(src[:nbytes], dst[:nbytes])
    assert int(dst[nbytes:].abs().sum()) == 0  # nothing past the end


def test_empty_kernel_runs():
    ref.empty(256, 256, _cs())
    torch.cuda.synchronize()


def test_weight_step_matches_definition():
    n, b = 4096, 6
    x, w = workloads.spectral_energy_inputs(n=n, batch=b, seed=5, wseed=6)
    y = torch.from_numpy(x).to(DEV)
    rows = torch.empty(b, device=DEV)
    ref.weight_energy(y.data_ptr(), torch.from_numpy(w).to(DEV).data_ptr(), rows.data_ptr(), n, b,
                      _cs())
    torch.cuda.synchronize()
    w2 = w.astype(np.float64) ** 2
    want_rows = np.sum(w2 * np.abs(x.astype(np.complex128)) ** 2, axis=1)
    assert np.max(np.abs(rows.cpu().numpy() - want_rows) / want_rows) <= 1e-5
    ok, worst, _, _ = metrics.gate(y.cpu().numpy(), 2 * w2 * x, x)
    assert ok, worst


def test_filter_step_and_unfused_chain_match_oracle():
    n, b = 4096, 5
    x = workloads.plain_normal(n, b, seed=8)
    h = workloads.complex_normal((n,), seed=9)
    xt, ht = torch.from_numpy(x).to(DEV), torch.from_numpy(h).to(DEV)
    y = sf.fft(xt)
    ref.filter_multiply(y.data_ptr(), ht.data_ptr(), n, b, _cs())
    z = sf.fft(y, inverse=True)
    torch.cuda.synchronize()
    ok, worst, _, ab = metrics.gate(z.cpu().numpy(), oracle.matched_filter(x, h), x)
    assert ok, (worst, ab)


@pytest.mark.parametrize("name", ref.timeline_variants())
@pytest.mark.parametrize("inverse", [False, True], ids=["fwd", "bwd"])
def test_timeline_transform_matches_oracle_and_stamps_are_ordered(name, inverse):
    by_name = {v["name"]: i for i, v in enumerate(sf.variants())}
    d = sf.fft_variant_describe(by_name[name])
    n, b = d["n"], 9
    waves = d["threads"] // 64
    x = workloads.plain_normal(n, b, seed=17)
    xt = torch.from_numpy(x).to(DEV)
    yt = torch.empty_like(xt)
    tw = torch.from_numpy(sf.fft_variant_twiddles(by_name[name])).to(DEV)
    st = torch.zeros(b * waves * 32, dtype=torch.int64, device=DEV)
    ref.timeline(name, xt.data_ptr(), yt.data_ptr(), tw.data_ptr(), b, inverse, st.data_ptr(), _cs())
    torch.cuda.synchronize()
    ok, worst, _, ab = metrics.gate(yt.cpu().numpy(), oracle.fft(x, inverse=inverse), x)
    assert ok, (worst, ab)
    # The stamps keep the scheduler from moving work across the marks, which
    # may change which products fuse into FMAs: the same arithmetic up to
    # rounding, not bit for bit.
    plain = sf.fft(xt, inverse=inverse, algorithm=sf.FFT_ALGO_SINGLE_PASS, variant=name)
    diff = (plain - yt).abs().amax(dim=1).cpu().numpy()  # per row
    assert np.all(diff <= 1e-5 * np.sqrt(np.sum(np.abs(x) ** 2, axis=1))), diff
    a = st.view(b * waves, 32).cpu().numpy()
    last = 2 * d["passes"] + 2
    for block in (a[:, :last + 1], a[:, 16:16 + last + 1]):
        assert np.all(block > 0)
        assert np.all(np.diff(block, axis=1) >= 0)
    assert np.all(a[:, last + 1:16] == 0)
