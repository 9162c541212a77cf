"""The LDS-poison debug build against the oracle.

libstockfft_poison.so is the transform library compiled with
STOCKFFT_LDS_POISON: every exchange buffer starts as NaNs and every slot is
overwritten with a NaN as soon as it has been read, so a barrier missing
between an exchange's writes and its reads, or between its reads and the
next exchange's writes, turns the output into NaNs.  Every single-pass
variant (plain, in-wave, streamed), the four-step splits up to 2^16, the
fused forward -> weight -> adjoint kernel and a ragged batch run through
the debug library's C ABI (its own ctypes handle; the product binding is
not involved) and must match the FP64 oracle to the usual gates.
"""
import ctypes
import os

import numpy as np
import pytest

import oracle
import paper_2603_27569_amd as sf
from paper_2603_27569_amd import _lib, metrics, workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

POISON = os.path.join(os.path.dirname(_lib.LIB_PATH), "libstockfft_poison.so")
DEV = torch.device("cuda:0")
SINGLE = [v for v in sf.variants() if v["kind"] == "single"]
FOUR = [v for v in sf.variants() if v["kind"] == "four_step" and v["n"] <= 1 << 16]


@pytest.fixture(scope="module")
def plib():
    if not os.path.exists(POISON):
        raise RuntimeError(f"{POISON} is missing: build the libraries first")
    lib = ctypes.CDLL(POISON)
    for name, (res, args) in _lib.SIGNATURES.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


def _stream():
    return torch.cuda.current_stream().cuda_stream


def _plan(lib, n, batch, direction, algorithm, variant):
    plan = ctypes.c_void_p()
    rc = lib.fft_plan_config(ctypes.byref(plan), n, batch, direction, algorithm,
                             variant.encode() if variant else None)
    assert rc == 0, _lib.STATUS.get(rc, rc)
    return plan


def _transform(lib, x, direction, algorithm, variant):
    batch, n = x.shape
    plan = _plan(lib, n, batch, direction, algorithm, variant)
    xt = torch.from_numpy(x).to(DEV)
    yt = torch.empty_like(xt)
    rc = lib.fft_exec(plan, xt.data_ptr(), yt.data_ptr(), _stream())
    torch.cuda.synchronize()
    assert rc == 0, _lib.STATUS.get(rc, rc)
    assert lib.fft_destroy(plan) == 0
    return yt.cpu().numpy()


def _gate(y, x, inverse=False):
    assert not np.isnan(y).any(), "NaN: an exchange slot was read before its write or after its poison"
    ok, worst, _, ab = metrics.gate(y, oracle.fft(x, inverse=inverse), x)
    assert ok, (worst, ab)


@pytest.mark.parametrize("v", SINGLE, ids=[v["name"] for v in SINGLE])
def test_single_pass_variant_under_lds_poison(plib, v):
    n = v["n"]
    if v["streamed"]:
        # a persistent shape's workgroups loop: one full round and a ragged second
        batch = torch.cuda.get_device_properties(0).multi_processor_count * v["streamed"] + 37
    else:
        batch = 3 * v["transforms_per_workgroup"] + 1
    x = workloads.plain_uniform(n, batch, seed=7 * n + batch)
    inverse = n % 3 == 1  # both directions across the lengths
    y = _transform(plib, x, sf.FFT_BACKWARD if inverse else sf.FFT_FORWARD, sf.FFT_ALGO_SINGLE_PASS,
                   v["name"])
    _gate(y, x, inverse)


@pytest.mark.parametrize("v", FOUR, ids=[v["name"] for v in FOUR])
def test_four_step_variant_under_lds_poison(plib, v):
    x = workloads.plain_uniform(v["n"], 3, seed=v["n"] + 5)
    _gate(_transform(plib, x, sf.FFT_FORWARD, sf.FFT_ALGO_FOUR_STEP, v["name"]), x)


def test_fused_forward_adjoint_under_lds_poison(plib):
    n, batch = 4096, 6
    xs, w = workloads.spectral_energy_inputs(n=n, batch=batch)
    plan = _plan(plib, n, batch, sf.FFT_FORWARD, sf.FFT_ALGO_AUTO, None)
    x = torch.from_numpy(xs).to(DEV)
    wt = torch.from_numpy(w).to(DEV)
    grad = torch.empty_like(x)
    rows = torch.empty(batch, device=DEV)
    total = torch.empty(1, device=DEV)
    rc = plib.fft_exec_spectral_energy(plan, x.data_ptr(), wt.data_ptr(), None, grad.data_ptr(),
                                       rows.data_ptr(), total.data_ptr(), _stream())
    torch.cuda.synchronize()
    assert rc == 0, _lib.STATUS.get(rc, rc)
    assert plib.fft_destroy(plan) == 0
    ref_rows, ref_grad = oracle.spectral_energy(xs, w)
    g = grad.cpu().numpy()
    assert not np.isnan(g).any()
    ok, rel, _ = metrics.grad_gate(g, ref_grad)
    assert ok, rel
    assert np.max(np.abs(rows.cpu().numpy() - ref_rows) / ref_rows) < 1e-5


def test_ragged_batch_under_lds_poison(plib):
    sizes, offs, data = workloads.ragged(count=40, seed=11)
    sz = (ctypes.c_int64 * len(sizes))(*[int(s) for s in sizes])
    plan = ctypes.c_void_p()
    assert plib.fft_plan_ragged(ctypes.byref(plan), sz, len(sizes), sf.FFT_FORWARD) == 0
    xin = torch.from_numpy(data).to(DEV)
    yout = torch.empty_like(xin)
    rc = plib.fft_exec_ragged(plan, xin.data_ptr(), yout.data_ptr(), _stream())
    torch.cuda.synchronize()
    assert rc == 0, _lib.STATUS.get(rc, rc)
    assert plib.fft_destroy_ragged(plan) == 0
    y = yout.cpu().numpy()
    for n in np.unique(sizes):
        idx = np.nonzero(sizes == n)[0]
        xr = np.stack([data[offs[i]:offs[i] + n] for i in idx])
        _gate(np.stack([y[offs[i]:offs[i] + n] for i in idx]), xr)
