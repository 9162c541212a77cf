"""Autotuner for the Stockham kernels on the current GPU.

For every transform length and batch bucket it times each compiled kernel
variant -- values per lane (hence the radix and lanes per transform),
transforms per workgroup, LDS padding, and for N >= 8192 the four-step
splits (for N > 16384 the only kind) -- through the C ABI, and keeps the
fastest.  The two fused kernels (the matched filter, and the forward ->
weight -> adjoint kernel with its loss total) and the transform with 16-bit
storage are tuned the same way, each on its own.  For the ragged persistent kernel
it picks one compiled shape per length by coordinate descent on a mixed
ragged batch.  The result is a JSON file that
``fft_tune_load`` (or the STOCKFFT_TUNE_CACHE environment variable) applies:

  {"arch": "gfx950", "cus": 256, "hip_runtime": ..., "entries": [
     {"n": 4096, "batch_min": 129, "batch_max": 1024,
      "variant": "n4096_e16_b1_p4_r16.16.16", "us": ..., "candidates": {...}}],
   "filter_entries": [...], "fused_entries": [...],
   "storage16_entries": [...],                          (same form)
   "ragged": [{"n": 4096, "shape": "ragged_n4096_e16", "batch_us": ...}]}

Each plain entry also records, per single-pass candidate, the registers,
scratch and LDS of its compiled kernel as the runtime reports them
("resources"), so a choice can be read against its occupancy and spills.

Timing: back-to-back launches over a ring of independent buffers larger
than the Infinity Cache, bracketed by HIP events on the launch stream; the
median of three repeats, each at least REPEAT_US of GPU time; candidates
within 3% of the best are timed again with three times the launches before
one is chosen.  Every variant computes the same transform (the
parity tests check each one against the FP64 reference), so the search is
on speed alone.

Usage: python -m paper_2603_27569_amd.tune [--out tune_gfx950.json] [--quick]
       python -m paper_2603_27569_amd.tune --run-variants N BATCH [--iters K]
         (no search: runs every variant of length N, K launches each, so that
         an external profiler can attribute counters to each variant)
       python -m paper_2603_27569_amd.tune --run-fused-variants N BATCH [--iters K]
         (the same for the fused forward -> weight -> adjoint kernel)
       python -m paper_2603_27569_amd.tune --merge-counters N BATCH CSV... [--iters K] --out FILE
         (attaches the counters of such a run under rocprofv3 --pmc, one CSV
         per counter pass, to FILE's entries for N at BATCH, per candidate)
"""
import argparse
import json
import math
import statistics
import sys

from . import (FFT_ALGO_FOUR_STEP, FFT_ALGO_SINGLE_PASS, FFT_FORWARD, FFT_IO_C16, Plan, RaggedPlan,
               fft_exec_io, fft_exec_matched_filter, fft_exec_spectral_energy, fft_ragged_shapes,
               fft_tune_clear_ragged, fft_tune_set_ragged, variants)

SIZES = (256, 512, 1024, 2048, 4096, 8192, 16384)
# Lengths with four-step splits only (plain transform; the fused kernels are
# single-pass); the timed batch is capped by MAX_BYTES per buffer.
SIZES_LARGE = tuple(1 << e for e in range(15, 21))
# Batch buckets: (batch_min, batch_max, representative batch timed).
BUCKETS = ((1, 64, 32), (65, 384, 256), (385, 768, 512), (769, 1536, 1024), (1537, 4096, 2048),
           (4097, 2 ** 62, 16384))
# Each timed repeat covers at least this much GPU time (launch counts adapt to
# the kernel's duration), and the candidates within CLOSE of the best are
# timed once more with FINAL_FACTOR times the launches before one is chosen.
REPEAT_US = 1500.0
CLOSE = 1.03
FINAL_FACTOR = 3
RING_BYTES = 1 << 30
MAX_BYTES = 2 << 30  # cap on one timed buffer


def _ring(torch, dev, n, batch):
    per = n * batch * 8
    k = max(2, math.ceil(RING_BYTES / (2 * per)))
    xs = [torch.randn(batch, n, dtype=torch.complex64, device=dev) for _ in range(k)]
    ys = [torch.empty_like(xs[0]) for _ in range(k)]
    return xs, ys


def _time(torch, stream, fn, iters, warmup=5, repeats=3):
    """Median over `repeats` of the per-launch time of back-to-back launches
    (microseconds).  `iters` is the least number of launches per repeat; it
    grows so that a repeat covers REPEAT_US of GPU time."""
    with torch.cuda.stream(stream):
        for i in range(warmup):
            fn(i)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    with torch.cuda.stream(stream):
        e0.record(stream)
        for i in range(5):
            fn(i)
        e1.record(stream)
    torch.cuda.synchronize()
    probe = max(e0.elapsed_time(e1) * 1e3 / 5, 1.0)
    iters = max(iters, min(2000, int(REPEAT_US / probe)))
    res = []
    for _ in range(repeats):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        with torch.cuda.stream(stream):
            e0.record(stream)
            for i in range(iters):
                fn(i)
            e1.record(stream)
        torch.cuda.synchronize()
        res.append(e0.elapsed_time(e1) * 1e3 / iters)
    return statistics.median(res)


def _pick(times, retime):
    """The fastest candidate, after re-timing every candidate within CLOSE of
    the first measurement's best (retime(name) returns a new time)."""
    best = min(times.values())
    close = [k for k, v in times.items() if v <= best * CLOSE]
    if len(close) > 1:
        for k in close:
            times[k] = retime(k)
    return min(times, key=times.get)


def filter_candidates(n):
    """Single-pass variants of length n that have the fused matched filter."""
    return [v["name"] for v in variants()
            if v["n"] == n and v["kind"] == "single" and v["fused_kernels"]]


def fused_candidates(n):
    """Single-pass variants of length n that have the fused forward -> weight ->
    adjoint kernel."""
    return [v["name"] for v in variants()
            if v["n"] == n and v["kind"] == "single" and v["fused_kernel"]]


def candidates(n):
    out = []
    for v in variants():
        if v["n"] != n:
            continue
        algo = FFT_ALGO_FOUR_STEP if v["kind"] == "four_step" else FFT_ALGO_SINGLE_PASS
        out.append((v["name"], algo))
    return out


def tune_plain(torch, dev, stream, sizes=SIZES, buckets=BUCKETS, iters=30, log=print):
    entries = []
    for n in sizes:
        for bmin, bmax, b in buckets:
            while n * b * 8 > MAX_BYTES and b > 1:
                b //= 2
            xs, ys = _ring(torch, dev, n, b)
            k = len(xs)
            times = {}
            res = {}
            cs = stream.cuda_stream
            algos = dict(candidates(n))

            def timed(name, factor=1):
                p = Plan(n, b, FFT_FORWARD, algos[name], name)
                if algos[name] == FFT_ALGO_SINGLE_PASS and name not in res:
                    r = p.describe().get("variant_resources")
                    if r:
                        res[name] = r
                t = _time(torch, stream,
                          lambda i: p.exec(xs[i % k].data_ptr(), ys[i % k].data_ptr(), cs),
                          iters * factor)
                p.close()
                return t

            for name in algos:
                times[name] = timed(name)
            best = _pick(times, lambda name: timed(name, FINAL_FACTOR))
            log(f"tune n={n} batch={b} -> {best} {times[best]:.2f} us")
            entries.append({"n": n, "batch_min": bmin, "batch_max": bmax, "variant": best,
                            "timed_batch": b, "us": round(times[best], 3),
                            "candidates": {k2: round(v, 3) for k2, v in times.items()},
                            "resources": res})
            del xs, ys
    return entries


def tune_filter(torch, dev, stream, sizes=SIZES, buckets=BUCKETS, iters=30, log=print):
    """The fused matched filter (forward, multiply by conj(h), inverse in one
    kernel) per length and batch bucket, over the single-pass variants."""
    entries = []
    for n in sizes:
        h = torch.randn(n, dtype=torch.complex64, device=dev)
        for bmin, bmax, b in buckets:
            while n * b * 8 > MAX_BYTES and b > 1:
                b //= 2
            xs, ys = _ring(torch, dev, n, b)
            k = len(xs)
            times = {}
            cs = stream.cuda_stream
            names = filter_candidates(n)

            def timed(name, factor=1):
                p = Plan(n, b, FFT_FORWARD, FFT_ALGO_SINGLE_PASS, name)
                t = _time(torch, stream,
                          lambda i: fft_exec_matched_filter(p.handle, xs[i % k].data_ptr(),
                                                            h.data_ptr(), ys[i % k].data_ptr(), cs),
                          iters * factor)
                p.close()
                return t

            for name in names:
                times[name] = timed(name)
            best = _pick(times, lambda name: timed(name, FINAL_FACTOR))
            log(f"tune filter n={n} batch={b} -> {best} {times[best]:.2f} us")
            entries.append({"n": n, "batch_min": bmin, "batch_max": bmax, "variant": best,
                            "timed_batch": b, "us": round(times[best], 3),
                            "candidates": {k2: round(v, 3) for k2, v in times.items()}})
            del xs, ys
    return entries


def tune_fused(torch, dev, stream, sizes=SIZES, buckets=BUCKETS, iters=30, log=print):
    """The fused forward -> weight -> adjoint kernel (gradient and loss total
    included) per length and batch bucket, over the single-pass variants."""
    entries = []
    for n in sizes:
        w = torch.rand(n, dtype=torch.float32, device=dev)
        total = torch.empty(1, dtype=torch.float32, device=dev)
        for bmin, bmax, b in buckets:
            while n * b * 8 > MAX_BYTES and b > 1:
                b //= 2
            xs, ys = _ring(torch, dev, n, b)
            k = len(xs)
            rows = torch.empty(b, dtype=torch.float32, device=dev)
            times = {}
            cs = stream.cuda_stream
            names = fused_candidates(n)

            def timed(name, factor=1):
                p = Plan(n, b, FFT_FORWARD, FFT_ALGO_SINGLE_PASS, name)
                t = _time(torch, stream,
                          lambda i: fft_exec_spectral_energy(
                              p.handle, xs[i % k].data_ptr(), w.data_ptr(), 0,
                              ys[i % k].data_ptr(), rows.data_ptr(), total.data_ptr(), cs),
                          iters * factor)
                p.close()
                return t

            for name in names:
                times[name] = timed(name)
            best = _pick(times, lambda name: timed(name, FINAL_FACTOR))
            log(f"tune fused n={n} batch={b} -> {best} {times[best]:.2f} us")
            entries.append({"n": n, "batch_min": bmin, "batch_max": bmax, "variant": best,
                            "timed_batch": b, "us": round(times[best], 3),
                            "candidates": {k2: round(v, 3) for k2, v in times.items()}})
            del xs, ys
    return entries


def tune_storage16(torch, dev, stream, sizes=SIZES, buckets=BUCKETS, iters=30, log=print):
    """The transform with binary16 storage (fft_exec_io, FFT_IO_C16) per
    length and batch bucket, over every single-pass variant.  The bfloat16
    format runs the same kernels with another conversion, so it shares the
    choice.  Half the bytes move, so the best shape can differ from FP32's."""
    entries = []
    for n in sizes:
        for bmin, bmax, b in buckets:
            while n * b * 4 > MAX_BYTES and b > 1:
                b //= 2
            k = max(2, math.ceil(RING_BYTES / (2 * n * b * 4)))
            xs = [torch.randn(b, n, 2, device=dev).to(torch.float16) for _ in range(k)]
            ys = [torch.empty_like(xs[0]) for _ in range(k)]
            times = {}
            cs = stream.cuda_stream
            names = [nm for nm, algo in candidates(n) if algo == FFT_ALGO_SINGLE_PASS]

            def timed(name, factor=1):
                p = Plan(n, b, FFT_FORWARD, FFT_ALGO_SINGLE_PASS, name)
                t = _time(torch, stream,
                          lambda i: fft_exec_io(p.handle, xs[i % k].data_ptr(), ys[i % k].data_ptr(),
                                                FFT_IO_C16, cs),
                          iters * factor)
                p.close()
                return t

            for name in names:
                times[name] = timed(name)
            best = _pick(times, lambda name: timed(name, FINAL_FACTOR))
            log(f"tune storage16 n={n} batch={b} -> {best} {times[best]:.2f} us")
            entries.append({"n": n, "batch_min": bmin, "batch_max": bmax, "variant": best,
                            "timed_batch": b, "us": round(times[best], 3),
                            "candidates": {k2: round(v, 3) for k2, v in times.items()}})
            del xs, ys
    return entries


def tune_ragged(torch, dev, stream, sizes=None, iters=20, sweeps=2, log=print):
    """Choose the ragged kernel's shape per length on a mixed ragged batch.

    The shapes interact (they share the persistent workgroups and the list
    schedule), so they are tuned together: coordinate descent over the lengths,
    each step timing every shape of one length with the others fixed.  The
    default batch is 2000 lengths drawn log-uniformly from 256..16384."""
    if sizes is None:
        from .workloads import ragged_sizes
        sizes = ragged_sizes()
    sizes = [int(s) for s in sizes]
    total = sum(sizes)
    k = max(2, math.ceil(RING_BYTES / (2 * total * 8)))
    xs = [torch.randn(total, dtype=torch.complex64, device=dev) for _ in range(k)]
    ys = [torch.empty_like(xs[0]) for _ in range(k)]
    cs = stream.cuda_stream
    present = sorted(set(sizes), reverse=True)
    choice = {n: fft_ragged_shapes(n)[0] for n in present}
    history = {n: {} for n in present}

    def timed():
        for n, sh in choice.items():
            fft_tune_set_ragged(n, sh)
        p = RaggedPlan(sizes)
        us = _time(torch, stream, lambda i: p.exec(xs[i % k].data_ptr(), ys[i % k].data_ptr(), cs),
                   iters)
        p.close()
        return us

    try:
        best_us = timed()
        for _ in range(sweeps):
            for n in present:
                for shape in fft_ragged_shapes(n):
                    if shape == choice[n]:
                        history[n][shape] = round(best_us, 3)
                        continue
                    old = choice[n]
                    choice[n] = shape
                    us = timed()
                    history[n][shape] = round(us, 3)
                    if us < best_us:
                        best_us = us
                    else:
                        choice[n] = old
                log(f"tune ragged n={n} -> {choice[n]} (batch {best_us:.2f} us)")
    finally:
        fft_tune_clear_ragged()
    del xs, ys
    return [{"n": n, "shape": choice[n], "batch_us": round(best_us, 3), "candidates": history[n]}
            for n in sorted(present)]


def run(out_path, quick=False, log=print):
    import torch
    dev = torch.device("cuda:0")
    stream = torch.cuda.Stream()
    props = torch.cuda.get_device_properties(dev)
    buckets = BUCKETS if not quick else ((1, 2 ** 62, 1024),)
    entries = tune_plain(torch, dev, stream, sizes=SIZES + SIZES_LARGE, buckets=buckets,
                         iters=10 if quick else 30, log=log)
    filters = tune_filter(torch, dev, stream, buckets=buckets, iters=10 if quick else 30, log=log)
    fused = tune_fused(torch, dev, stream, buckets=buckets, iters=10 if quick else 30, log=log)
    storage16 = tune_storage16(torch, dev, stream, buckets=buckets, iters=10 if quick else 30,
                               log=log)
    ragged = tune_ragged(torch, dev, stream, iters=5 if quick else 20, sweeps=1 if quick else 2,
                         log=log)
    doc = {"arch": props.gcnArchName.split(":")[0], "cus": props.multi_processor_count,
           "hip_runtime": getattr(torch.version, "hip", None), "entries": entries,
           "filter_entries": filters, "fused_entries": fused, "storage16_entries": storage16,
           "ragged": ragged}
    with open(out_path, "w") as f:
        json.dump(doc, f, indent=1)
    return doc


def run_variants(n, batch, iters=10, log=print):
    """Runs each compiled variant of length n (forward, batch rows) `iters`
    times on one pair of buffers and synchronises; no timing, no choice."""
    import torch
    dev = torch.device("cuda:0")
    stream = torch.cuda.Stream()
    x = torch.randn(batch, n, dtype=torch.complex64, device=dev)
    y = torch.empty_like(x)
    with torch.cuda.stream(stream):
        y.copy_(x)  # a plain device copy of known size, to scale byte counters by
    torch.cuda.synchronize()
    for v in variants():
        if v["n"] != n:
            continue
        algo = FFT_ALGO_SINGLE_PASS if v["kind"] == "single" else FFT_ALGO_FOUR_STEP
        p = Plan(n, batch, FFT_FORWARD, algo, v["name"])
        for _ in range(iters):
            p.exec(x.data_ptr(), y.data_ptr(), stream.cuda_stream)
        torch.cuda.synchronize()
        p.close()
        log(f"ran {v['name']} x{iters}")


def run_fused_variants(n, batch, iters=10, log=print):
    """The same for the fused forward -> weight -> adjoint kernel (with its
    loss total): every variant of length n that has it, `iters` calls each."""
    import torch
    dev = torch.device("cuda:0")
    stream = torch.cuda.Stream()
    x = torch.randn(batch, n, dtype=torch.complex64, device=dev)
    w = torch.rand(n, device=dev)
    g = torch.empty_like(x)
    rows = torch.empty(batch, device=dev)
    total = torch.empty(1, device=dev)
    torch.cuda.synchronize()
    for name in fused_candidates(n):
        p = Plan(n, batch, FFT_FORWARD, FFT_ALGO_SINGLE_PASS, name)
        for _ in range(iters):
            fft_exec_spectral_energy(p.handle, x.data_ptr(), w.data_ptr(), 0, g.data_ptr(),
                                     rows.data_ptr(), total.data_ptr(), stream.cuda_stream)
        torch.cuda.synchronize()
        p.close()
        log(f"ran fused {name} x{iters}")


def variant_dispatch_counters(csv_paths, n, iters):
    """Per-variant counter medians from rocprofv3 counter-collection CSV files
    (`--pmc ... --output-format csv`) of a `--run-variants n BATCH --iters
    iters` run, one file per counter pass.  run_variants launches each variant
    of length n `iters` times in variants() order (a four-step variant two
    kernels per launch), so the library's own dispatches, taken in dispatch
    order, split into consecutive runs that map one to one onto the variants;
    every other dispatch (the calibration copy, fills and copies of plan
    creation) is left out.  Returns {variant: {counter: median}}, with
    `<counter>_per_wave` added for SQ_ counters when SQ_WAVES was collected."""
    import csv
    names = [(v["name"], 1 if v["kind"] == "single" else 2) for v in variants() if v["n"] == n]
    out = {name: {} for name, _ in names}
    for path in csv_paths:
        disp = {}
        with open(path) as f:
            for r in csv.DictReader(f):
                if "stockfft::" not in r["Kernel_Name"]:
                    continue
                d = disp.setdefault(int(r["Dispatch_Id"]), {"kernel": r["Kernel_Name"], "c": {}})
                d["c"][r["Counter_Name"]] = float(r["Counter_Value"])
        seq = [disp[k] for k in sorted(disp)]
        need = sum(k for _, k in names) * iters
        if len(seq) != need:
            raise ValueError(f"{path}: {len(seq)} library dispatches, expected {need} "
                             f"({len(names)} variants of length {n} x {iters} launches)")
        pos = 0
        for name, k in names:
            run = seq[pos:pos + k * iters]
            pos += k * iters
            kinds = {d["kernel"] for d in run[:k]}
            if any(d["kernel"] != run[i % k]["kernel"] for i, d in enumerate(run)) or len(kinds) != k:
                raise ValueError(f"{path}: the dispatches of {name} are not one repeated launch")
            for c in run[0]["c"]:
                out[name][c] = statistics.median(sum(d["c"][c] for d in run[i:i + k])
                                                 for i in range(0, len(run), k))
    for name, cs in out.items():
        waves = cs.get("SQ_WAVES")
        if waves:
            for c in [c for c in cs if c.startswith("SQ_") and c != "SQ_WAVES"]:
                cs[c + "_per_wave"] = round(cs[c] / waves, 2)
    return out


def merge_counters(doc, n, batch, counters):
    """Attach per-candidate counters to the plain entries of length n whose
    bucket holds `batch` (entry["counters"][variant])."""
    hit = 0
    for e in doc["entries"]:
        if e["n"] == n and e["batch_min"] <= batch <= e["batch_max"]:
            e["counters"] = {"batch": batch, "by_variant": counters}
            hit += 1
    if not hit:
        raise ValueError(f"no tuned entry of length {n} holds batch {batch}")
    return doc


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--out", default="tune_gfx950.json")
    ap.add_argument("--quick", action="store_true")
    ap.add_argument("--run-variants", nargs=2, type=int, metavar=("N", "BATCH"))
    ap.add_argument("--run-fused-variants", nargs=2, type=int, metavar=("N", "BATCH"))
    ap.add_argument("--iters", type=int, default=10)
    ap.add_argument("--merge-counters", nargs="+", metavar="N BATCH CSV",
                    help="attach per-variant counter medians of a profiled --run-variants N BATCH "
                         "run (rocprofv3 counter-collection CSV files) to the --out tune file")
    a = ap.parse_args(argv)
    log = lambda *x: print(*x, file=sys.stderr, flush=True)  # noqa: E731
    if a.merge_counters:
        n, batch, paths = int(a.merge_counters[0]), int(a.merge_counters[1]), a.merge_counters[2:]
        with open(a.out) as f:
            doc = json.load(f)
        merge_counters(doc, n, batch, variant_dispatch_counters(paths, n, a.iters))
        with open(a.out, "w") as f:
            json.dump(doc, f, indent=1)
        return 0
    if a.run_variants:
        run_variants(a.run_variants[0], a.run_variants[1], a.iters, log=log)
        return 0
    if a.run_fused_variants:
        run_fused_variants(a.run_fused_variants[0], a.run_fused_variants[1], a.iters, log=log)
        return 0
    run(a.out, a.quick, log=log)
    return 0


if __name__ == "__main__":
    sys.exit(main())
