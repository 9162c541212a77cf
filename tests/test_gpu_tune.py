"""The autotuner end to end on a restricted search, and plans honouring it."""
import json

import numpy as np
import pytest

import oracle
import paper_2603_27569_amd as sf
from paper_2603_27569_amd import metrics, tune, workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def test_tuner_restricted_search_and_load(tmp_path):
    dev = torch.device("cuda:0")
    s = torch.cuda.Stream()
    entries = tune.tune_plain(torch, dev, s, sizes=(256, 8192), buckets=((1, 2 ** 62, 64),),
                              iters=3, log=lambda *a: None)
    assert {e["n"] for e in entries} == {256, 8192}
    for e in entries:
        assert e["variant"] in e["candidates"]
        assert e["us"] == min(e["candidates"].values())
        singles = {v["name"] for v in sf.variants() if v["kind"] == "single" and v["n"] == e["n"]}
        assert set(e["resources"]) == singles
        for r in e["resources"].values():
            assert 0 < r["vgprs"] <= 512 and r["scratch_bytes_per_lane"] >= 0 and r["lds_bytes"] > 0
    path = tmp_path / "tune.json"
    path.write_text(json.dumps({"arch": "gfx950", "entries": entries, "ragged": []}))
    sf.fft_tune_clear()
    try:
        sf.fft_tune_load(str(path))
        for e in entries:
            assert sf.fft_tune_query(e["n"], 64) == e["variant"]
            x = workloads.plain_normal(e["n"], 5, seed=1)
            p = sf.Plan(e["n"], 5)
            d = p.describe()
            chosen = d.get("four_step", d["variant"])["name"]
            assert chosen == e["variant"]
            xt = torch.from_numpy(x).to(dev)
            y = torch.empty_like(xt)
            p.exec(xt.data_ptr(), y.data_ptr(), torch.cuda.current_stream().cuda_stream)
            torch.cuda.synchronize()
            ok, worst, _, _ = metrics.gate(y.cpu().numpy(), oracle.fft(x), x)
            assert ok, worst
            p.close()
    finally:
        sf.fft_tune_clear()


def test_fused_tuner_restricted_search():
    dev = torch.device("cuda:0")
    s = torch.cuda.Stream()
    entries = tune.tune_fused(torch, dev, s, sizes=(1024,), buckets=((1, 2 ** 62, 64),),
                              iters=3, log=lambda *a: None)
    assert [e["n"] for e in entries] == [1024]
    e = entries[0]
    names = {v["name"] for v in sf.variants()
             if v["kind"] == "single" and v["n"] == 1024 and v["fused_kernel"]}
    assert set(e["candidates"]) == names
    assert e["variant"] in names and e["us"] == min(e["candidates"].values())


def test_storage16_tuner_restricted_search_and_plan_choice(tmp_path):
    dev = torch.device("cuda:0")
    s = torch.cuda.Stream()
    entries = tune.tune_storage16(torch, dev, s, sizes=(2048,), buckets=((1, 2 ** 62, 64),),
                                  iters=3, log=lambda *a: None)
    assert [e["n"] for e in entries] == [2048]
    e = entries[0]
    names = {v["name"] for v in sf.variants() if v["kind"] == "single" and v["n"] == 2048}
    assert set(e["candidates"]) == names
    assert e["variant"] in names and e["us"] == min(e["candidates"].values())
    # A plan made without a variant runs the 16-bit transform with the
    # 16-bit table's choice, which need not be the FP32 one.
    other = next(nm for nm in sorted(names) if nm != sf.fft_tune_query(2048, 64))
    path = tmp_path / "tune.json"
    path.write_text(json.dumps({"arch": "gfx950", "storage16_entries": [
        {"n": 2048, "batch_min": 1, "batch_max": 2 ** 62, "variant": other}]}))
    sf.fft_tune_clear()
    try:
        sf.fft_tune_load(str(path))
        assert sf.fft_tune_query_storage16(2048, 64) == other
        for direction in (sf.FFT_FORWARD, sf.FFT_BACKWARD):
            p = sf.Plan(2048, 64, direction)
            d = p.describe()
            assert d["storage16_variant"] == other and d["variant"]["name"] != other
            x = workloads.complex_normal((64, 2048), seed=5)
            stored, xv = workloads.to_storage(x, "f16")
            xin = torch.from_numpy(np.ascontiguousarray(stored)).to(dev)
            y = torch.empty_like(xin)
            sf.fft_exec_io(p.handle, xin.data_ptr(), y.data_ptr(), sf.FFT_IO_C16, 0)
            torch.cuda.synchronize()
            yh = y.cpu().numpy().astype(np.float64)
            ref = oracle.fft(xv, inverse=direction == sf.FFT_BACKWARD)
            ok, worst, _, _ = metrics.gate_storage(yh[..., 0] + 1j * yh[..., 1], ref, xv, "f16")
            assert ok, worst
            p.close()
    finally:
        sf.fft_tune_clear()


def test_ragged_shape_tuner():
    dev = torch.device("cuda:0")
    s = torch.cuda.Stream()
    before = sf.fft_tune_query_ragged(4096)
    sizes = workloads.ragged_sizes(count=120, seed=3)
    out = tune.tune_ragged(torch, dev, s, sizes=sizes, iters=2, sweeps=1, log=lambda *a: None)
    assert [o["n"] for o in out] == sorted(set(int(v) for v in sizes))
    for o in out:
        assert o["shape"] in sf.fft_ragged_shapes(o["n"])
    assert sf.fft_tune_query_ragged(4096) == before  # the tuner leaves no state behind


def test_stale_tune_files_are_ignored(tmp_path):
    """A file tuned for another architecture or on another CU count leaves the
    table as it was; a file for this device is applied."""
    props = torch.cuda.get_device_properties(0)
    arch = props.gcnArchName.split(":")[0]
    cus = props.multi_processor_count
    sf.fft_tune_clear()
    try:
        before = sf.fft_tune_query(2048, 5)
        other = next(v["name"] for v in sf.variants()
                     if v["kind"] == "single" and v["n"] == 2048 and v["name"] != before)
        entries = [{"n": 2048, "batch_min": 1, "batch_max": 10 ** 9, "variant": other}]
        path = tmp_path / "tune.json"
        for doc in ({"arch": "gfx942", "cus": cus, "entries": entries},
                    {"arch": arch, "cus": cus + 1, "entries": entries},
                    {"arch": arch, "cus": cus // 4, "entries": entries}):
            path.write_text(json.dumps(doc))
            with pytest.raises(sf.StockfftError):
                sf.fft_tune_load(str(path))
            assert sf.fft_tune_query(2048, 5) == before
        path.write_text(json.dumps({"arch": arch, "cus": cus, "entries": entries}))
        sf.fft_tune_load(str(path))
        assert sf.fft_tune_query(2048, 5) == other
    finally:
        sf.fft_tune_clear()


def test_plan_log_names_the_tuned_choices(monkeypatch, capfd):
    """STOCKFFT_LOG prints each plan's choices on stderr; unset, nothing."""
    sf.fft_tune_clear()
    monkeypatch.setenv("STOCKFFT_LOG", "1")
    p = sf.Plan(4096, 32, sf.FFT_FORWARD)
    p.close()
    err = capfd.readouterr().err
    line = next(ln for ln in err.splitlines() if ln.startswith("stockfft: plan n=4096 batch=32"))
    assert f"variant={sf.fft_tune_query(4096, 32)} " in line
    assert "algorithm=single_pass" in line and "source=tuned" in line
    assert f"storage16={sf.fft_tune_query_storage16(4096, 32)} " in line
    monkeypatch.setenv("STOCKFFT_LOG", "0")
    sf.Plan(4096, 32, sf.FFT_FORWARD).close()
    assert "stockfft: plan" not in capfd.readouterr().err
