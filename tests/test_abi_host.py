"""Host-side checks of the C ABI: exported symbols, argument validation
(returned before any HIP call), twiddle tables and plan structure.  These
run without a GPU."""
import ctypes
import json
import os
import re
import subprocess

import numpy as np
import pytest

import paper_2603_27569_amd as sf
from paper_2603_27569_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "stockfft.h")
GOLDEN = os.path.join(ROOT, "tests", "golden", "paper_tables.json")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(fft_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    L = _lib.lib()
    names = _declared()
    assert len(names) >= 20
    for n in names:
        assert hasattr(L, n), n
    # the binding declares exactly the header's entry points
    assert sorted(_lib.SIGNATURES) == names
    out = subprocess.run(["nm", "-D", "--defined-only", _lib.LIB_PATH], capture_output=True,
                         text=True).stdout
    exported = set(re.findall(r" T (fft_[a-z0-9_]+)$", out, flags=re.M))
    assert set(names) <= exported


def test_lds_poison_debug_library_exports_the_same_abi():
    """libstockfft_poison.so (the transform library built with
    STOCKFFT_LDS_POISON, for the tests only) exports the header's entry
    points, like the product library."""
    path = os.path.join(os.path.dirname(_lib.LIB_PATH), "libstockfft_poison.so")
    out = subprocess.run(["nm", "-D", "--defined-only", path], capture_output=True,
                         text=True).stdout
    exported = set(re.findall(r" T (fft_[a-z0-9_]+)$", out, flags=re.M))
    assert set(_declared()) <= exported


def test_status_strings_and_version():
    for code in range(13):
        assert sf.fft_status_string(code)
    assert sf.fft_version() >= 10000


def _plan_rc(n, batch, direction, algo=0, variant=None, null_out=False):
    h = ctypes.c_void_p(12345)
    ptr = None if null_out else ctypes.byref(h)
    rc = _lib.lib().fft_plan_config(ptr, n, batch, direction, algo,
                                    variant.encode() if variant else None)
    return rc, h.value


@pytest.mark.parametrize("n", [0, 1, 128, 255, 257, 3000, 3 * 2 ** 15, 2 ** 21, -4096])
def test_invalid_size_rejected_before_device(n):
    rc, h = _plan_rc(n, 1, -1)
    assert rc == _lib.CODES["FFT_INVALID_SIZE"] and h is None


@pytest.mark.parametrize("batch", [0, -1, 2 ** 62])
def test_invalid_batch(batch):
    rc, h = _plan_rc(4096, batch, -1)
    assert rc == _lib.CODES["FFT_INVALID_BATCH"] and h is None


@pytest.mark.parametrize("d", [0, 2, -2])
def test_invalid_direction(d):
    assert _plan_rc(4096, 1, d)[0] == _lib.CODES["FFT_INVALID_DIRECTION"]


def test_invalid_algorithm_and_variant_names():
    assert _plan_rc(4096, 1, -1, algo=7)[0] == _lib.CODES["FFT_INVALID_ARGUMENT"]
    assert _plan_rc(4096, 1, -1, variant="nope")[0] == _lib.CODES["FFT_INVALID_ARGUMENT"]
    assert _plan_rc(4096, 1, -1, variant="n256_e16_b16_p4_r16.16")[0] == _lib.CODES["FFT_INVALID_ARGUMENT"]
    assert _plan_rc(4096, 1, -1, algo=2)[0] == _lib.CODES["FFT_UNSUPPORTED"]
    assert _plan_rc(4096, 1, -1, null_out=True)[0] == _lib.CODES["FFT_INVALID_POINTER"]


def test_exec_and_destroy_reject_bad_handles():
    L = _lib.lib()
    assert L.fft_exec(None, None, None, None) == _lib.CODES["FFT_INVALID_PLAN"]
    assert L.fft_exec(ctypes.c_void_p(0xdead0), None, None, None) == _lib.CODES["FFT_INVALID_PLAN"]
    assert L.fft_destroy(None) == 0
    assert L.fft_destroy(ctypes.c_void_p(0xdead0)) == _lib.CODES["FFT_INVALID_PLAN"]
    assert L.fft_exec_spectral_energy(None, None, None, None, None, None, None, None) == \
        _lib.CODES["FFT_INVALID_PLAN"]
    assert L.fft_exec_matched_filter(None, None, None, None, None) == _lib.CODES["FFT_INVALID_PLAN"]
    assert L.fft_exec_ragged(None, None, None, None) == _lib.CODES["FFT_INVALID_PLAN"]
    assert L.fft_exec_ragged_direct(None, None, None, None) == _lib.CODES["FFT_INVALID_PLAN"]
    assert L.fft_destroy_ragged(None) == 0


def test_ragged_plan_validation():
    L = _lib.lib()
    h = ctypes.c_void_p()
    arr = (ctypes.c_int64 * 3)(256, 1000, 4096)
    assert L.fft_plan_ragged(ctypes.byref(h), arr, 3, -1) == _lib.CODES["FFT_INVALID_SIZE"]
    arr = (ctypes.c_int64 * 2)(256, 4096)
    assert L.fft_plan_ragged(ctypes.byref(h), arr, 0, -1) == _lib.CODES["FFT_INVALID_BATCH"]
    assert L.fft_plan_ragged(ctypes.byref(h), arr, 2, 5) == _lib.CODES["FFT_INVALID_DIRECTION"]
    assert L.fft_plan_ragged(ctypes.byref(h), None, 2, -1) == _lib.CODES["FFT_INVALID_POINTER"]
    assert L.fft_plan_ragged(None, arr, 2, -1) == _lib.CODES["FFT_INVALID_POINTER"]


def test_tune_file_with_four_step_and_ragged_entries(tmp_path):
    sf.fft_tune_clear()
    sf.fft_tune_clear_ragged()
    try:
        p = tmp_path / "t.json"
        p.write_text(json.dumps({"arch": "gfx950", "cus": 256, "entries": [
            {"n": 16384, "batch_min": 1, "batch_max": 8, "variant": "fs16384_4x4096", "us": 1.0},
            {"n": 16384, "batch_min": 9, "batch_max": 10 ** 12, "variant": "n16384_e32_b1_p4_r16.16.16.4"},
            {"n": 512, "batch_min": 1, "batch_max": 10 ** 12, "variant": "n512_e8_b4_p4_r8.8.8",
             "candidates": {"n512_e4_b2_p4_r4.4.4.4.2": 3.0}}],
            "ragged": [{"n": 2048, "shape": "ragged_n2048_e16", "us": 2.0}]}))
        sf.fft_tune_load(str(p))
        assert sf.fft_tune_query(16384, 4) == "fs16384_4x4096"
        assert sf.fft_tune_query(16384, 1024) == "n16384_e32_b1_p4_r16.16.16.4"
        assert sf.fft_tune_query(512, 77) == "n512_e8_b4_p4_r8.8.8"
        assert sf.fft_tune_query_ragged(2048) == "ragged_n2048_e16"
        sf.fft_tune_set(8192, 1, 10, "fs8192_2x4096")
        assert sf.fft_tune_query(8192, 3) == "fs8192_2x4096"
    finally:
        sf.fft_tune_clear()
        sf.fft_tune_clear_ragged()


def test_builtin_table_is_the_shipped_tuner_output():
    """The library's built-in choices equal the autotuner's MI355X result
    shipped with the package (tune_gfx950.json)."""
    sf.fft_tune_clear()
    sf.fft_tune_clear_ragged()
    doc = json.load(open(os.path.join(ROOT, "paper_2603_27569_amd", "tune_gfx950.json")))
    assert doc["arch"] == "gfx950"
    for e in doc["entries"]:
        for b in (e["batch_min"], e["timed_batch"], min(e["batch_max"], 10 ** 9)):
            assert sf.fft_tune_query(e["n"], b) == e["variant"], (e["n"], b)
    for r in doc["ragged"]:
        assert sf.fft_tune_query_ragged(r["n"]) == r["shape"]
    for e in doc.get("filter_entries", []):
        for b in (e["batch_min"], e["timed_batch"], min(e["batch_max"], 10 ** 9)):
            assert sf.fft_tune_query_filter(e["n"], b) == e["variant"], (e["n"], b)
    assert doc.get("fused_entries")
    for e in doc["fused_entries"]:
        for b in (e["batch_min"], e["timed_batch"], min(e["batch_max"], 10 ** 9)):
            assert sf.fft_tune_query_fused(e["n"], b) == e["variant"], (e["n"], b)
    # every shipped single-pass choice was recorded with its kernel's
    # resources, and none of them spills
    for e in doc["entries"]:
        if e["n"] <= 16384 and not e["variant"].startswith("fs"):
            r = e["resources"][e["variant"]]
            assert r["scratch_bytes_per_lane"] == 0 and 0 < r["vgprs"] <= 512, e["variant"]
    assert doc.get("storage16_entries")
    for e in doc["storage16_entries"]:
        for b in (e["batch_min"], e["timed_batch"], min(e["batch_max"], 10 ** 9)):
            assert sf.fft_tune_query_storage16(e["n"], b) == e["variant"], (e["n"], b)


def test_shipped_table_buckets_tile_every_batch():
    """Per length, the shipped entries (plain and matched filter) cover batch 1
    to the maximum without gaps or overlaps, follow the tuner's bucket list,
    and each was timed inside its own bucket."""
    from paper_2603_27569_amd import tune
    doc = json.load(open(os.path.join(ROOT, "paper_2603_27569_amd", "tune_gfx950.json")))
    lows = [b[0] for b in tune.BUCKETS]
    for key in ("entries", "filter_entries", "fused_entries", "storage16_entries"):
        by_n = {}
        for e in doc[key]:
            by_n.setdefault(e["n"], []).append(e)
        sizes = set(tune.SIZES) | (set(tune.SIZES_LARGE) if key == "entries" else set())
        assert set(by_n) == sizes, key
        for n, es in by_n.items():
            es = sorted(es, key=lambda e: e["batch_min"])
            assert [e["batch_min"] for e in es] == lows, (key, n)
            assert es[-1]["batch_max"] >= 2 ** 62, (key, n)
            for a, b2 in zip(es, es[1:]):
                assert a["batch_max"] + 1 == b2["batch_min"], (key, n)
            for e in es:
                assert e["variant"] in e["candidates"], (key, n)
                assert e["us"] == min(e["candidates"].values()), (key, n)
                # timed inside the bucket (large lengths cap the timed batch)
                assert e["timed_batch"] <= e["batch_max"], (key, n)


def test_ragged_shape_tuning_api():
    sf.fft_tune_clear_ragged()
    builtin = {n: sf.fft_tune_query_ragged(n) for n in (256, 512, 1024, 2048, 4096, 8192, 16384)}
    try:
        for n in builtin:
            shapes = sf.fft_ragged_shapes(n)
            assert len(shapes) == 2 and builtin[n] in shapes
            assert all(sh.startswith(f"ragged_n{n}_") for sh in shapes)
            for sh in shapes:
                sf.fft_tune_set_ragged(n, sh)
                assert sf.fft_tune_query_ragged(n) == sh
        with pytest.raises(sf.StockfftError):
            sf.fft_tune_set_ragged(16384, sf.fft_ragged_shapes(256)[0])
        with pytest.raises(sf.StockfftError):
            sf.fft_tune_set_ragged(300, sf.fft_ragged_shapes(256)[0])
    finally:
        sf.fft_tune_clear_ragged()
    assert {n: sf.fft_tune_query_ragged(n) for n in builtin} == builtin


def test_no_device_reported_cleanly():
    try:
        import torch
        if torch.cuda.is_available():
            pytest.skip("a device is present")
    except Exception:
        pass
    rc, h = _plan_rc(4096, 8, -1)
    assert rc == _lib.CODES["FFT_NO_DEVICE"] and h is None


# ---------------------------------------------------------------- variants

def _variants():
    return sf.variants()


def test_variant_inventory():
    vs = _variants()
    singles = [v for v in vs if v["kind"] == "single"]
    fours = [v for v in vs if v["kind"] == "four_step"]
    assert {v["n"] for v in singles} == {256, 512, 1024, 2048, 4096, 8192, 16384}
    assert {v["n"] for v in fours} == {2 ** e for e in range(13, 21)}
    for v in fours:
        assert v["n1"] * v["n2"] == v["n"]
        assert v["two_level_twiddles"] == (v["n"] > 16384)
    names = [v["name"] for v in vs]
    assert len(set(names)) == len(names)
    for v in singles:
        assert int(np.prod(v["radices"])) == v["n"]
        assert v["lanes_per_transform"] * v["values_per_lane"] == v["n"]
        assert all(v["values_per_lane"] % r == 0 for r in v["radices"])
        assert v["threads"] == v["lanes_per_transform"] * v["transforms_per_workgroup"] <= 1024
        chunk = v["n"] // v["exchange_rounds"]
        pad = (chunk >> v["pad_log2"]) if v["pad_log2"] > 0 else 0
        assert v["lds_layout"] == ("pad" if v["pad_log2"] > 0 else "xor" if v["pad_log2"] < 0 else "none")
        bufs = 2 if v["double_buffered"] else 1
        assert v["lds_bytes"] == v["transforms_per_workgroup"] * bufs * (chunk + pad) * 8
        assert v["lds_bytes"] <= 160 * 1024  # gfx950 LDS per workgroup
        c = v["exchange_rounds"]
        if v["wave_exchange"]:  # exchanges after passes 0 and 2 in registers: one LDS exchange
            assert v["n"] == 4096 and v["radices"] == [8, 8, 8, 8] and c == 1
            assert v["barriers"] == 1 and v["fused_kernels"]
            assert v["wave_members"] in (1, 2)
            assert v["values_per_lane"] == 8 * v["wave_exchange"] * v["wave_members"]
        elif v["double_buffered"]:  # one barrier per exchange, whole-transform rounds
            assert c == 1 and v["barriers"] == v["passes"] - 1
        else:
            assert v["barriers"] == (2 * c * (v["passes"] - 1) - 1 if v["passes"] > 1 else 0)
        if c > 1:  # every exchange pass splits evenly into the rounds
            assert all((v["values_per_lane"] // r) % c == 0 for r in v["radices"][:-1])


def test_paper_table_v_radix4_shapes():
    """The radix-4 variants are the paper's Table V kernels: N/4 lanes, the
    printed pass counts, and the printed exchange-buffer size."""
    g = json.load(open(GOLDEN))["table_v_multisize_radix4"]["rows"]
    by_n = {v["n"]: v for v in _variants() if v["kind"] == "single" and v["values_per_lane"] == 4}
    for row in g:
        v = by_n[row["n"]]
        assert v["lanes_per_transform"] == row["threads"]
        assert v["radices"].count(4) == row["radix4_passes"]
        assert v["radices"].count(2) == row["radix2_tail"]
        assert v["n"] * 8 == row["tg_kib"] * 1024


def test_paper_table_iv_stage_counts():
    """Stages at N=4096 per radix (Table IV); our barrier count is one fewer
    than the paper's 2(stages-1) because the first exchange write needs no
    preceding barrier."""
    g = json.load(open(GOLDEN))["table_iv_radix_analysis_n4096"]["rows"]
    by_r = {}
    for v in _variants():
        if v["kind"] == "single" and v["n"] == 4096 and len(set(v["radices"])) == 1:
            by_r.setdefault(v["radices"][0], v)
    for row in g:
        if row["radix"] not in by_r:
            continue
        v = by_r[row["radix"]]
        assert v["passes"] == row["stages"]
        assert v["barriers"] == row["barriers"] - 1
    assert {4, 8, 16} <= set(by_r)


def test_paper_four_step_splits_present():
    g = json.load(open(GOLDEN))["four_step_splits"]["rows"]
    fours = {(v["n"], v["n1"], v["n2"]) for v in _variants() if v["kind"] == "four_step"}
    for row in g:
        assert (row["n"], row["n1"], row["n2"]) in fours


def _exact_roots(m, L):
    return np.exp(-2j * np.pi * m / L)


def _ulp_err(tab, exact):
    exact = np.asarray(exact)
    er = np.abs(tab.real.astype(np.float64) - exact.real)
    ei = np.abs(tab.imag.astype(np.float64) - exact.imag)
    ur = np.spacing(np.abs(exact.real).astype(np.float32)).astype(np.float64)
    ui = np.spacing(np.abs(exact.imag).astype(np.float32)).astype(np.float64)
    return max(np.max(er / ur), np.max(ei / ui))


def _stockham_expect(radices, paired):
    """Exact table entries of a Stockham plan; None marks a pad (must be 0).
    Plain layout [r - 1][k] = W^{k r}; paired layout (passes of radix >= 4)
    [q][k][h] = W^{k (2q + 1 + h)}."""
    expect = []
    ns = radices[0]
    for r_p in radices[1:]:
        L = ns * r_p
        if paired and r_p >= 4:
            for q in range(r_p // 2):
                for k in range(ns):
                    for h in range(2):
                        r = 2 * q + 1 + h
                        expect.append(_exact_roots(k * r, L) if r < r_p else None)
        else:
            for r in range(1, r_p):
                for k in range(ns):
                    expect.append(_exact_roots(k * r, L))
        ns *= r_p
    return expect


def test_twiddle_tables_rounded_once_from_fp64():
    """Every table entry is W_L^m rounded once to FP32: within half an ulp of
    the exact root (plus FP64 evaluation slack); pads of the paired layout are
    exactly zero."""
    vs = _variants()
    seen_paired = False
    for i, v in enumerate(vs):
        tab = sf.fft_variant_twiddles(i)
        if v["kind"] == "single":
            radices = v["radices"]
            paired = v["paired_twiddles"]
            seen_paired |= paired
        else:
            sub = next(s for s in vs if s["name"] == v["sub_variant"])
            radices = sub["radices"]
            paired = sub["paired_twiddles"]
        expect = _stockham_expect(radices, paired)
        pads = np.array([e is None for e in expect] + [False] * (len(tab) - len(expect)))
        if pads.shape == tab.shape and pads.any():
            assert np.all(tab[pads] == 0), v["name"]
            tab = tab[~pads]
        expect = [e for e in expect if e is not None]
        if v["kind"] == "four_step" and not v["two_level_twiddles"]:
            N = v["n"]
            for n1 in range(1, v["n1"]):
                for k2 in range(v["n2"]):
                    expect.append(_exact_roots(n1 * k2, N))
        elif v["kind"] == "four_step":
            # lo[j] = W_N^j (j < 2^s), hi[j] = W_N^(j 2^s) (j < N / 2^s), W_N1^j (j < N1)
            N = v["n"]
            s = (N.bit_length() - 1) // 2
            expect += [_exact_roots(j, N) for j in range(2 ** s)]
            expect += [_exact_roots(j << s, N) for j in range(N >> s)]
            expect += [_exact_roots(j, v["n1"]) for j in range(v["n1"])]
            if v["sub2_variant"]:  # the second stage's own N1-point table
                sub2 = next(s for s in vs if s["name"] == v["sub2_variant"])
                assert sub2["n"] == v["n1"] and not sub2["paired_twiddles"]
                expect += _stockham_expect(sub2["radices"], False)
        expect = np.array(expect)
        assert tab.shape == expect.shape, v["name"]
        assert _ulp_err(tab, expect) <= 0.5 + 1e-6, v["name"]
    assert seen_paired


def test_tune_table_set_query_load(tmp_path):
    sf.fft_tune_clear()
    try:
        base = sf.fft_tune_query(4096, 256)
        assert base.startswith("n4096_")
        sf.fft_tune_set(4096, 1, 100, "n4096_e8_b1_p4_r8.8.8.8")
        assert sf.fft_tune_query(4096, 50) == "n4096_e8_b1_p4_r8.8.8.8"
        assert sf.fft_tune_query(4096, 256) == base
        with pytest.raises(sf.StockfftError):
            sf.fft_tune_set(4096, 1, 10, "n256_e16_b16_p4_r16.16")
        p = tmp_path / "tune.json"
        p.write_text(json.dumps({"arch": "gfx950", "entries": [
            {"n": 2048, "batch_min": 1, "batch_max": 10 ** 9, "variant": "n2048_e8_b1_p4_r8.8.8.4"},
            {"n": 2048, "batch_min": 1, "batch_max": 10, "variant": "bogus"}],
            "filter_entries": [
            {"n": 1024, "batch_min": 1, "batch_max": 10 ** 9, "variant": "n1024_e4_b1_p4_r4.4.4.4.4"},
            {"n": 1024, "batch_min": 1, "batch_max": 10, "variant": "n2048_e8_b1_p4_r8.8.8.4"}],
            "fused_entries": [
            {"n": 512, "batch_min": 1, "batch_max": 10 ** 9, "variant": "n512_e4_b2_p4_r4.4.4.4.2"},
            {"n": 512, "batch_min": 1, "batch_max": 10, "variant": "bogus"}],
            "storage16_entries": [
            {"n": 512, "batch_min": 1, "batch_max": 10 ** 9, "variant": "n512_e16_b2_p4_r16.16.2"},
            {"n": 512, "batch_min": 1, "batch_max": 10, "variant": "n1024_e4_b1_p4_r4.4.4.4.4"}]}))
        sf.fft_tune_load(str(p))
        assert sf.fft_tune_query_fused(512, 5) == "n512_e4_b2_p4_r4.4.4.4.2"
        # the entry naming another length's variant is skipped
        assert sf.fft_tune_query_storage16(512, 5) == "n512_e16_b2_p4_r16.16.2"
        with pytest.raises(sf.StockfftError):
            sf.fft_tune_query_storage16(32768, 5)
        with pytest.raises(sf.StockfftError):
            sf.fft_tune_query_fused(32768, 5)
        assert sf.fft_tune_query(2048, 5) == "n2048_e8_b1_p4_r8.8.8.4"
        assert sf.fft_tune_query_filter(1024, 5) == "n1024_e4_b1_p4_r4.4.4.4.4"
        with pytest.raises(sf.StockfftError):
            sf.fft_tune_query_filter(32768, 5)  # no single-pass kernel at that length
        with pytest.raises(sf.StockfftError):
            sf.fft_tune_load(str(tmp_path / "missing.json"))
        bad = tmp_path / "bad.json"
        for text in ('{"entries": [', '{"entries": [{"n": 2048,}]}', "[1, 2", '{"a" 1}'):
            bad.write_text(text)
            with pytest.raises(sf.StockfftError):
                sf.fft_tune_load(str(bad))
        assert sf.fft_tune_query(2048, 5) == "n2048_e8_b1_p4_r8.8.8.4"
    finally:
        sf.fft_tune_clear()


def test_tune_file_malformed_documents_and_fields(tmp_path):
    """Tune files outside JSON's grammar are refused whole; entries whose
    numbers are not integers in range are skipped; a malformed "arch" or
    "cus" refuses the file (no device needed for these checks)."""
    sf.fft_tune_clear()
    try:
        base = sf.fft_tune_query(2048, 5)
        base16 = sf.fft_tune_query_storage16(2048, 5)
        bad = tmp_path / "bad.json"
        docs = [
            '{"entries": [{"n": 2048, "batch_min": NaN, "variant": "x"}]}',  # not JSON
            '{"entries": [{"n": 2048, "batch_min": Infinity}]}',
            '{"entries": [{"n": 2048, "batch_min": 1e400}]}',  # overflows double
            '{"entries": [{"n": 0x800}]}',
            '{"entries": [{"n": +2048}]}',
            '{"entries": [{"n": 2048.}]}',
            '{"arch": "gfx9\\u00zz"}',  # bad escape digits
            '{"arch": "gfx9\\u12"}',  # truncated escape
            '{"arch": "gfx\\q950"}',  # not a JSON escape
            '{"entries": [' * 100 + ']' * 100 + '}',  # 100-deep nesting
            '{"entries": [{"n": 2048, "variant": "n2048_e8_b1_p4_r8.8.8.4"}',  # truncated
            '{"arch": ""}',  # empty arch
            '{"arch": ":sramecc+"}',
            '{"arch": 950}',
            '{"cus": 0}', '{"cus": -256}', '{"cus": 2.5}', '{"cus": "256"}',
        ]
        for text in docs:
            bad.write_text(text)
            with pytest.raises(sf.StockfftError) as e:
                sf.fft_tune_load(str(bad))
            assert e.value.name == "FFT_INVALID_ARGUMENT", text
        good = "n2048_e16_b1_p4_r16.16.8"
        entries = [
            {"n": 2048, "batch_min": -5, "batch_max": 10, "variant": good},
            {"n": 2048, "batch_min": 0, "batch_max": 10, "variant": good},
            {"n": 2048, "batch_min": 1.5, "batch_max": 10, "variant": good},
            {"n": 2048, "batch_min": 9, "batch_max": 3, "variant": good},
            {"n": 2048.5, "batch_min": 1, "batch_max": 10, "variant": good},
            {"n": -2048, "batch_min": 1, "batch_max": 10, "variant": good},
            {"n": 2048, "batch_min": 1, "batch_max": -1e30, "variant": good},
            {"n": 2048, "batch_min": "1", "batch_max": 10, "variant": good},
        ]
        p = tmp_path / "skip.json"
        p.write_text(json.dumps({"arch": "gfx950:sramecc+:xnack-", "cus": 256, "entries": entries,
                                 "filter_entries": entries, "fused_entries": entries,
                                 "storage16_entries": entries,
                                 "ragged": [{"n": 2048.5, "shape": "ragged_n2048_e16"}]}))
        sf.fft_tune_load(str(p))  # loads, every entry skipped
        assert sf.fft_tune_query(2048, 5) == base
        assert sf.fft_tune_query_storage16(2048, 5) == base16
        # a huge batch_max saturates (the tuner's unbounded bucket is 2^62)
        p.write_text(json.dumps({"entries": [
            {"n": 2048, "batch_min": 1, "batch_max": 1e19, "variant": good}]}))
        sf.fft_tune_load(str(p))
        assert sf.fft_tune_query(2048, 5) == good
        assert sf.fft_tune_query(2048, 2 ** 62) == good
    finally:
        sf.fft_tune_clear()
        sf.fft_tune_clear_ragged()


def test_reference_library_exports_its_header():
    from paper_2603_27569_amd import reference
    header = os.path.join(ROOT, "include", "stockref.h")
    text = re.sub(r"/\*.*?\*/", "", open(header).read(), flags=re.S)
    names = sorted(set(re.findall(r"\b(ref_[a-z_]+)\s*\(", text)))
    assert sorted(reference.SIGNATURES) == names
    L = reference.lib()
    for n in names:
        assert hasattr(L, n), n
    out = subprocess.run(["nm", "-D", "--defined-only", reference.LIB_PATH], capture_output=True,
                         text=True).stdout
    assert set(names) <= set(re.findall(r" T (ref_[a-z_]+)$", out, flags=re.M))
    # the transform library does not carry the references
    out = subprocess.run(["nm", "-D", "--defined-only", _lib.LIB_PATH], capture_output=True,
                         text=True).stdout
    assert not re.findall(r" T (ref_[a-z_]+)$", out, flags=re.M)
    assert reference.timeline_variants()[0] == sf.fft_tune_query(4096, 256)  # the headline shape


def test_reference_calls_reject_bad_arguments_before_any_device_call():
    from paper_2603_27569_amd import reference as R
    L = R.lib()
    codes = _lib.CODES
    vp = ctypes.c_void_p
    assert L.ref_empty(0, 64, None) == codes["FFT_INVALID_ARGUMENT"]
    assert L.ref_empty(1, 2048, None) == codes["FFT_INVALID_ARGUMENT"]
    assert L.ref_copy_rows(None, vp(64), 4096, 1, 256, None) == codes["FFT_INVALID_POINTER"]
    assert L.ref_copy_rows(vp(64), vp(1 << 30), 4096, 1, 128, None) == codes["FFT_INVALID_ARGUMENT"]
    assert L.ref_copy_rows(vp(68), vp(1 << 30), 4096, 1, 256, None) == codes["FFT_MISALIGNED"]
    assert L.ref_copy_rows(vp(64), vp(64 + 8), 4096, 1, 256, None) == codes["FFT_OVERLAP"]
    assert L.ref_copy_wide(vp(64), vp(1 << 30), 24, None) == codes["FFT_INVALID_ARGUMENT"]
    assert L.ref_copy_wide(vp(72), vp(1 << 30), 32, None) == codes["FFT_MISALIGNED"]
    assert L.ref_weight_energy(vp(64), vp(64), vp(64), 300, 1, None) == codes["FFT_INVALID_ARGUMENT"]
    assert L.ref_filter_multiply(vp(64), None, 256, 1, None) == codes["FFT_INVALID_POINTER"]
    assert L.ref_lds_exchange(0, 1, vp(64), None) == codes["FFT_INVALID_ARGUMENT"]
    assert L.ref_lds_exchange(1, -1, vp(64), None) == codes["FFT_INVALID_ARGUMENT"]
    assert L.ref_lds_exchange(1, 1, None, None) == codes["FFT_INVALID_POINTER"]
    assert L.ref_lds_exchange(1, 1, vp(66), None) == codes["FFT_MISALIGNED"]
    assert L.ref_timeline(b"nope", vp(64), vp(1 << 30), vp(64), 1, 0, vp(64), None) == \
        codes["FFT_INVALID_ARGUMENT"]
    assert L.ref_timeline(b"n4096_e16_b1_px_r16.16.16_db", vp(64), vp(1 << 30), vp(64), 1, 2,
                          vp(64), None) == codes["FFT_INVALID_ARGUMENT"]


def test_tuner_maps_profiled_dispatches_to_variants(tmp_path):
    """tune --merge-counters: the library's dispatches of a profiled
    --run-variants run, in dispatch order, map one to one onto the variants
    of the length (other kernels -- the calibration copy, fills -- left out),
    and each variant gets the median of its launches."""
    from paper_2603_27569_amd import tune
    n, iters = 2048, 3
    vs = [(v["name"], 1 if v["kind"] == "single" else 2) for v in _variants() if v["n"] == n]
    path = tmp_path / "p1_counter_collection.csv"
    rows = ["Dispatch_Id,Kernel_Name,Counter_Name,Counter_Value"]
    d = 0

    def emit(kernel, values):
        nonlocal d
        d += 1
        for c, val in values.items():
            rows.append(f'{d},"{kernel}",{c},{val}')

    emit("at::copy_kernel", {"SQ_WAVES": 9, "SQ_INSTS_VALU": 1})
    for i, (name, k) in enumerate(vs):
        emit("__amd_rocclr_fillBuffer", {"SQ_WAVES": 1, "SQ_INSTS_VALU": 5})
        for j in range(iters):
            for part in range(k):
                emit(f"void stockfft::k_stockham<{name}, {part}>(stockfft::c32 const*)",
                     {"SQ_WAVES": 4, "SQ_INSTS_VALU": 100 * i + 10 * j + part})
    path.write_text("\n".join(rows) + "\n")
    got = tune.variant_dispatch_counters([str(path)], n, iters)
    assert set(got) == {name for name, _ in vs}
    for i, (name, k) in enumerate(vs):
        # launches j = 0, 1, 2 sum their k kernels: median at j = 1
        want = k * (100 * i + 10) + sum(range(k))
        assert got[name]["SQ_INSTS_VALU"] == want
        assert got[name]["SQ_WAVES"] == 4 * k
        assert got[name]["SQ_INSTS_VALU_per_wave"] == round(want / (4 * k), 2)
    doc = {"entries": [{"n": n, "batch_min": 65, "batch_max": 384}, {"n": n, "batch_min": 385,
                                                                       "batch_max": 768}]}
    tune.merge_counters(doc, n, 256, got)
    assert doc["entries"][0]["counters"]["by_variant"] == got and "counters" not in doc["entries"][1]
    # a run that does not match the variant list is refused
    path.write_text("\n".join(rows[:-3]) + "\n")
    with pytest.raises(ValueError):
        tune.variant_dispatch_counters([str(path)], n, iters)


def test_bench_names_compiled_variants():
    """The shapes bench.py names in its exchange-tier comparison are compiled
    variants of N = 4096 with the layouts the comparison's labels state."""
    import bench
    by = {v["name"]: v for v in _variants()}
    for label, name in bench.EXCHANGE_TIERS:
        v = by[name]
        assert v["n"] == 4096 and v["radices"] == [8, 8, 8, 8], name
        assert bool(v["wave_exchange"]) == label.startswith("in_wave"), name
