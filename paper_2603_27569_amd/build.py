"""Build the HIP libraries in-tree for gfx950.

Every translation unit under csrc/ is compiled with hipcc (in parallel) and
linked into paper_2603_27569_amd/libstockfft.so; refsrc/ (measurement
references, not part of the transform path) into libstockref.so.  The same
csrc/ sources compiled with STOCKFFT_LDS_POISON make the debug library
libstockfft_poison.so (every LDS exchange slot overwritten with a NaN once
read, to expose a missing barrier), which only the tests load.  Packed FP32
instructions are disabled for all device code.
"""
import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libstockfft.so")
POISON_LIB = os.path.join(HERE, "libstockfft_poison.so")
REFSRC = os.path.join(HERE, "refsrc")
REFLIB = os.path.join(HERE, "libstockref.so")
BUILD_DIR = os.path.join(ROOT, "_build")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-I", os.path.join(ROOT, "include"),
]


# Per-file options: the matrix-core kernels keep their accumulators in
# ordinary VGPRs (no copies out of the accumulation registers per product).
EXTRA = {"mma.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form"]}


def sources():
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC)
                  if f.endswith((".hip", ".cpp")))


def _compile(src, poison=False):
    sub = os.path.basename(os.path.dirname(src)) + ("_poison" if poison else "")
    obj = os.path.join(BUILD_DIR, sub + "_" + os.path.basename(src) + ".o")
    lang = ["-x", "hip"] if src.endswith(".cpp") else []
    defs = ["-DSTOCKFFT_LDS_POISON"] if poison else []
    cmd = [HIPCC, *FLAGS, *defs, *EXTRA.get(os.path.basename(src), []), *lang, "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return obj


def _link(objs, lib):
    tmp = lib + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    subprocess.run(cmd, check=True)
    os.replace(tmp, lib)


def build(jobs=None):
    """Compiles libstockfft.so (csrc/) and the measurement references
    libstockref.so (refsrc/, which the transform library never loads)."""
    os.makedirs(BUILD_DIR, exist_ok=True)
    srcs = sources()
    refs = [os.path.join(REFSRC, f) for f in sorted(os.listdir(REFSRC)) if f.endswith(".hip")]
    jobs = jobs or min(2 * len(srcs) + len(refs), max(1, min(8, os.cpu_count() or 1)))
    units = [(f, False) for f in srcs + refs] + [(f, True) for f in srcs]
    # the largest translation units first, so the pool's tail is short
    order = sorted(range(len(units)), key=lambda i: -os.path.getsize(units[i][0]))
    with cf.ThreadPoolExecutor(jobs) as ex:
        done = dict(zip(order, ex.map(lambda i: _compile(*units[i]), order)))
    objs = [done[i] for i in range(len(units))]
    n = len(srcs)
    _link(objs[:n], LIB)
    _link(objs[n:n + len(refs)], REFLIB)
    _link(objs[n + len(refs):], POISON_LIB)
    return LIB


if __name__ == "__main__":
    print(build())
    sys.exit(0)
