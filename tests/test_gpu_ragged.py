"""Ragged batches: the persistent kernel (its hipGraph and its plain launch)
against the FP64 oracle, transform by transform, plus graph re-use with new
pointers, per-size shape choices and the list schedule's edge cases."""
import numpy as np
import pytest

import oracle
import paper_2603_27569_amd as sf
from paper_2603_27569_amd import metrics, workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _check_ragged(y, x, sizes, inverse=False):
    offs = np.concatenate([[0], np.cumsum(sizes)[:-1]]).astype(np.int64)
    worst = 0.0
    for s in np.unique(sizes):
        idx = np.nonzero(sizes == s)[0]
        xr = np.stack([x[offs[i]:offs[i] + s] for i in idx])
        yr = np.stack([y[offs[i]:offs[i] + s] for i in idx])
        ok, w, _, ab = metrics.gate(yr, oracle.fft(xr, inverse=inverse), xr)
        assert ok, (int(s), w, ab)
        worst = max(worst, w)
    return worst


def _run(plan, x, graph=True):
    xt = torch.from_numpy(x).to(DEV)
    y = torch.full_like(xt, complex(float("nan"), float("nan")))
    sf.ragged_fft(xt, plan, out=y, graph=graph)
    torch.cuda.synchronize()
    return y


@pytest.mark.parametrize("graph", [True, False], ids=["graph", "direct"])
@pytest.mark.parametrize("inverse", [False, True], ids=["fwd", "bwd"])
def test_ragged_2000_matches_oracle(inverse, graph):
    sizes, offs, data = workloads.ragged()
    plan = sf.RaggedPlan(sizes, sf.FFT_BACKWARD if inverse else sf.FFT_FORWARD)
    y = _run(plan, data, graph).cpu().numpy()
    worst = _check_ragged(y, data, sizes, inverse)
    print(f"ragged 2000 inverse={inverse} graph={graph}: worst rel-RMS {worst:.3e}", flush=True)
    plan.close()


def test_ragged_graph_and_direct_launch_agree_bitwise():
    sizes, _, data = workloads.ragged(count=400, seed=31)
    plan = sf.RaggedPlan(sizes)
    a = _run(plan, data, graph=True)
    b = _run(plan, data, graph=False)
    c = _run(plan, data, graph=True)
    assert torch.equal(a, b) and torch.equal(a, c)
    plan.close()


def test_ragged_more_workgroups_than_tasks_and_many_tasks():
    # 3 transforms: fewer tasks than workgroups (most workgroups idle).
    # 20000 transforms of 256: many tasks per workgroup.
    for sizes in ([16384, 8192, 256], [256] * 20000):
        sizes = np.array(sizes, dtype=np.int64)
        x = workloads.complex_normal((int(sizes.sum()),), seed=int(sizes.size))
        plan = sf.RaggedPlan(sizes)
        _check_ragged(_run(plan, x).cpu().numpy(), x, sizes)
        plan.close()


@pytest.mark.parametrize("sizes", [
    [4096],
    [256],
    [16384, 256],
    [256] * 130 + [512] * 3,
    [8192, 512, 16384, 256, 1024, 2048, 4096, 4096, 256],
], ids=["one4096", "one256", "two", "partial_tasks", "mixed"])
def test_ragged_small_sets(sizes):
    sizes = np.array(sizes, dtype=np.int64)
    x = workloads.complex_normal((int(sizes.sum()),), seed=len(sizes))
    plan = sf.RaggedPlan(sizes)
    _check_ragged(_run(plan, x).cpu().numpy(), x, sizes)
    plan.close()


def test_ragged_graph_reuse_new_pointers():
    sizes, _, data = workloads.ragged(count=300, seed=77)
    plan = sf.RaggedPlan(sizes)
    x1 = torch.from_numpy(data).to(DEV)
    x2 = x1 * (0.5 - 0.25j)
    outs = []
    # Same pointers twice, then new pointers, then the first ones again: every
    # launch must do the whole batch, into the buffers of that call.
    for xin in (x1, x1, x2, x1):
        y = torch.full_like(x1, complex(float("nan"), 0.0))
        sf.ragged_fft(xin, plan, out=y)
        outs.append(y)
    torch.cuda.synchronize()
    assert torch.equal(outs[0], outs[1]) and torch.equal(outs[0], outs[3])
    _check_ragged(outs[0].cpu().numpy(), data, sizes)
    _check_ragged(outs[2].cpu().numpy(), x2.cpu().numpy(), sizes)
    # in place
    z = x1.clone()
    sf.ragged_fft(z, plan, out=z)
    torch.cuda.synchronize()
    assert torch.equal(z, outs[0])
    plan.close()


def test_ragged_every_shape_choice():
    sizes, _, data = workloads.ragged(count=200, seed=5)
    try:
        for n in workloads.SIZES:
            for shape in sf.fft_ragged_shapes(n):
                sf.fft_tune_set_ragged(n, shape)
        plan = sf.RaggedPlan(sizes)
        _check_ragged(_run(plan, data).cpu().numpy(), data, sizes)
        plan.close()
    finally:
        sf.fft_tune_clear_ragged()


def test_ragged_plain_comparator_matches():
    sizes, offs, data = workloads.ragged(count=120, seed=9)
    plan = sf.RaggedPlan(sizes)
    xt = torch.from_numpy(data).to(DEV)
    ins, outs = [], []
    for s in workloads.SIZES:
        idx = np.nonzero(sizes == s)[0]
        if len(idx) == 0:
            ins.append(None)
            outs.append(None)
            continue
        ins.append(torch.cat([xt[int(offs[i]):int(offs[i]) + int(s)] for i in idx]))
        outs.append(torch.empty_like(ins[-1]))
    plan.exec_plain([t.data_ptr() if t is not None else 0 for t in ins],
                    [t.data_ptr() if t is not None else 0 for t in outs],
                    torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    for s, t_in, t_out in zip(workloads.SIZES, ins, outs):
        if t_in is None:
            continue
        xr = t_in.cpu().numpy().reshape(-1, s)
        ok, w, _, _ = metrics.gate(t_out.cpu().numpy().reshape(-1, s), oracle.fft(xr), xr)
        assert ok, (s, w)
    plan.close()


def test_ragged_exec_errors():
    plan = sf.RaggedPlan([256, 512])
    buf = torch.zeros(2048, dtype=torch.complex64, device=DEV)
    L = sf._lib.lib()
    import ctypes
    vp = ctypes.c_void_p
    base = buf.data_ptr()
    assert L.fft_exec_ragged(vp(plan.handle), vp(base + 4), vp(base + 8 * 1024), None) == sf.CODES["FFT_MISALIGNED"]
    assert L.fft_exec_ragged(vp(plan.handle), vp(base), vp(base + 8), None) == sf.CODES["FFT_OVERLAP"]
    assert L.fft_exec_ragged_direct(vp(plan.handle), vp(base + 4), vp(base + 8 * 1024), None) == \
        sf.CODES["FFT_MISALIGNED"]
    assert L.fft_exec_ragged_direct(vp(plan.handle), vp(base), vp(base + 8), None) == sf.CODES["FFT_OVERLAP"]
    h = plan.handle
    plan.close()
    assert L.fft_exec_ragged(vp(h), vp(base), vp(base), None) == sf.CODES["FFT_INVALID_PLAN"]
    assert L.fft_exec_ragged_direct(vp(h), vp(base), vp(base), None) == sf.CODES["FFT_INVALID_PLAN"]
    torch.cuda.synchronize()
