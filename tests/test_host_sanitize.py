"""Host code under the address and undefined-behaviour sanitizers.

Builds, with g++/gcc and -fsanitize=address,undefined (host code only; no
GPU code is compiled here), the FP64 oracle with a driver that runs its
pins, and a harness of the library's host-only parsers and twiddle-table
builders (csrc/json_lite.hpp, csrc/twiddles.hpp), then runs them over
well-formed, malformed and randomly mutated tune files.  Any sanitizer
report fails the run (-fno-sanitize-recover=all).
"""
import json
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests", "sanitize")
CSRC = os.path.join(ROOT, "paper_2603_27569_amd", "csrc")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
       "-g", "-O1"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
           UBSAN_OPTIONS="print_stacktrace=1")

pytestmark = pytest.mark.skipif(shutil.which("g++") is None or shutil.which("gcc") is None,
                                reason="needs gcc and g++")


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, env=ENV, timeout=300, **kw)
    assert r.returncode == 0, f"{' '.join(cmd)}\n{r.stdout}\n{r.stderr}"
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr
    return r.stdout


@pytest.fixture(scope="module")
def harness(tmp_path_factory):
    d = tmp_path_factory.mktemp("san")
    exe = str(d / "host_harness")
    _run(["g++", "-std=c++17", *SAN, "-I", CSRC, os.path.join(HERE, "host_harness.cpp"),
          "-o", exe])
    return exe


def test_oracle_pins_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_driver")
    _run(["gcc", "-std=c99", *SAN, "-fno-fast-math", "-ffp-contract=off",
          os.path.join(HERE, "oracle_driver.c"), os.path.join(ROOT, "oracle", "fft_oracle.c"),
          "-o", exe, "-lm"])
    assert "oracle pins clean" in _run([exe])


def test_twiddle_builders_under_sanitizers(harness):
    out = _run([harness, "twiddles"])
    assert out.strip().endswith(", 0 bad"), out


MALFORMED = [
    '{"entries": [',  # truncated
    '{"entries": [{"n": 2048,}]}',
    '{"a" 1}',
    '{"n": NaN}', '{"n": -Infinity}', '{"n": 1e400}', '{"n": 0x10}', '{"n": 1.}', '{"n": .5}',
    '{"n": -}', '{"n": 1e}', '{"s": "\\u12"}', '{"s": "\\u00zz"}', '{"s": "\\q"}', '{"s": "abc',
    '{"s": "abc\\',
    '[' * 100 + ']' * 100,  # nesting deeper than the reader's 64 levels
    '{"a": 1} trailing',
    '',
]
WELLFORMED = [
    '{"n": -0.5e-3, "m": 12345678901234567890, "s": "\\u0041\\"\\\\\\/\\n", "t": true, "f": false, '
    '"z": null, "a": [], "o": {}}',
    '[' * 60 + ']' * 60,
]


def test_json_reader_on_malformed_and_wellformed(harness, tmp_path):
    paths = []
    for i, text in enumerate(MALFORMED + WELLFORMED):
        p = tmp_path / f"doc{i}.json"
        p.write_text(text)
        paths.append(str(p))
    got = _run([harness, "parse", *paths]).split()
    assert got == ["fail"] * len(MALFORMED) + ["ok"] * len(WELLFORMED)


def test_json_reader_fuzzed_tune_file(harness, tmp_path):
    with open(os.path.join(ROOT, "paper_2603_27569_amd", "tune_gfx950.json")) as f:
        doc = json.load(f)
    doc["entries"] = doc["entries"][:6]  # a short document keeps the run fast
    p = tmp_path / "tune.json"
    p.write_text(json.dumps(doc, indent=1))
    assert "ok" == _run([harness, "parse", str(p)]).strip()
    out = _run([harness, "fuzz", "20260101", "4000", str(p)])
    assert "of 4000 mutations parsed" in out
