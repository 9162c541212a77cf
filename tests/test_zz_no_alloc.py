"""fft_exec_spectral_energy_noalloc, called through the C ABI: the same
gradient and loss total as fft_exec_spectral_energy on two calls in a row
(the second with a smaller input), bit for bit, and the oracle's gates; the
batch limit and the required loss_total are enforced."""
import ctypes

import numpy as np
import pytest

import oracle
import paper_2603_27569_amd as sf
from paper_2603_27569_amd import _lib, metrics, workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _run_both(n, batch, seed, want_grad=True):
    x, w = workloads.spectral_energy_inputs(n=n, batch=batch, seed=seed, wseed=seed + 1)
    xt, wt = torch.from_numpy(x).to(DEV), torch.from_numpy(w).to(DEV)
    p = sf.Plan(n, batch, sf.FFT_FORWARD, sf.FFT_ALGO_SINGLE_PASS)
    cs = torch.cuda.current_stream().cuda_stream
    g_ref = torch.empty_like(xt)
    rows = torch.empty(batch, device=DEV)
    tot_ref = torch.empty(1, device=DEV)
    sf.fft_exec_spectral_energy(p.handle, xt.data_ptr(), wt.data_ptr(), 0,
                                g_ref.data_ptr() if want_grad else 0, rows.data_ptr(),
                                tot_ref.data_ptr(), cs)
    g = torch.full_like(xt, float("nan"))
    tot = torch.full((1,), float("nan"), device=DEV)
    L = _lib.lib()
    vp = ctypes.c_void_p
    rc = L.fft_exec_spectral_energy_noalloc(vp(p.handle), vp(xt.data_ptr()), vp(wt.data_ptr()),
                                            None, vp(g.data_ptr()) if want_grad else None,
                                            vp(tot.data_ptr()), vp(cs))
    assert rc == 0, sf.fft_status_string(rc)
    torch.cuda.synchronize()
    p.close()
    return x, w, g, g_ref, tot, tot_ref


def test_noalloc_matches_existing_entry_two_calls_smaller_second():
    for n, batch, seed in ((4096, 512, 71), (1024, 40, 73)):
        x, w, g, g_ref, tot, tot_ref = _run_both(n, batch, seed)
        assert torch.equal(tot, tot_ref)
        assert torch.equal(g, g_ref)
        ref_rows, ref_grad = oracle.spectral_energy(x, w)
        ok, worst, ab = metrics.grad_gate(g.cpu().numpy(), ref_grad)
        assert ok, (n, batch, worst, ab)
        assert abs(float(tot.cpu()[0]) - ref_rows.sum()) / ref_rows.sum() <= 1e-5


def test_noalloc_loss_only_and_repeat():
    totals = []
    for want in (False, True, False):
        _, _, _, _, tot, tot_ref = _run_both(2048, 300, 75, want_grad=want)
        assert torch.equal(tot, tot_ref)
        totals.append(float(tot.cpu()[0]))
    assert totals[0] == totals[1] == totals[2]


def test_noalloc_rejects_oversize_batch_and_missing_total():
    L = _lib.lib()
    vp = ctypes.c_void_p
    codes = sf.CODES
    p = sf.Plan(256, (1 << 20) + 1, sf.FFT_FORWARD, sf.FFT_ALGO_SINGLE_PASS)
    # arguments are checked before any device work: no buffers needed
    assert L.fft_exec_spectral_energy_noalloc(vp(p.handle), vp(64), vp(64), None, None, vp(64),
                                              None) == codes["FFT_INVALID_ARGUMENT"]
    p.close()
    q = sf.Plan(256, 4, sf.FFT_FORWARD, sf.FFT_ALGO_SINGLE_PASS)
    assert L.fft_exec_spectral_energy_noalloc(vp(q.handle), vp(64), vp(64), None, None, None,
                                              None) == codes["FFT_INVALID_POINTER"]
    q.close()
    b = sf.Plan(256, 4, sf.FFT_BACKWARD, sf.FFT_ALGO_SINGLE_PASS)
    assert L.fft_exec_spectral_energy_noalloc(vp(b.handle), vp(64), vp(64), None, None, vp(64),
                                              None) == codes["FFT_UNSUPPORTED"]
    b.close()
