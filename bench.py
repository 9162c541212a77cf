"""Benchmark of the batched FP32 c2c FFT on one MI355X.

Headline workload (one step): the forward and the backward transform of a
batch of 256 rows of N = 4096 complex64 values (the paper's Table VI shape),
inputs resident in HBM.  Throughput follows the paper's convention
(Section VI-A): 5 N log2 N flops per transform; HBM traffic is counted
algorithmically as 16 N bytes per transform (read + write, complex64).

Timing: W untimed warmup steps, then K timed steps bracketed by device
synchronisation, measured with HIP events recorded on the stream the
kernels are launched on.  Every step uses the next slot of a ring of
independent buffers whose total footprint exceeds 1 GiB, so the 256 MB
Infinity Cache cannot serve the inputs from an earlier step.

Beside the headline line the JSON carries: the roofline of the dominant
kernel, the FP64 oracle timed on the host cores (a baseline, not a target),
and the comparisons the paper's method implies (fused forward+adjoint vs
the plain chain, fused range compression vs its unfused chain, ragged
persistent launch vs per-size plain launches, four-step vs single-pass at
8192/16384, the four-step at 2^16 and 2^20, 16-bit storage against FP32
storage with vector-ALU and with matrix-core DFTs, a same-footprint copy
kernel).  The accuracy figures reported
here are against numpy's FP64 FFT (an independent library routine); the
parity tests against the oracle are the test suite's job.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-compare]
                       [--skip-cpu] [--sweep] [--timeline]
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

N_HEAD, B_HEAD = 4096, 256
RING_BYTES = 1 << 30
HBM_PEAK_GBS = 8000.0
PAPER_CONTEXT = {"gflops": 138.45, "us_per_fft": 1.78, "hardware": "Apple M1 GPU (8 cores)",
                 "vendor_baseline_gflops": 107.0, "source": "Table VI"}
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_fft_n4096_b256.json")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash():
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2603_27569_amd", "csrc")
    for f in ("stockham.hpp", "kernels.hpp", "wavex.hpp", "variants_4096.hip"):
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def ref_fft(np, x, inverse=False):
    """numpy's FP64 FFT along the last axis, unscaled in both directions."""
    a = np.asarray(x).astype(np.complex128)
    return np.fft.ifft(a, axis=-1, norm="forward") if inverse else np.fft.fft(a, axis=-1)


def median_of(T, fn, iters, warmup, trials=5):
    """Median over `trials` event-timed runs of `iters` launches (seconds per launch)."""
    ts = sorted(T.run(fn, iters, warmup) / iters for _ in range(trials))
    return ts[len(ts) // 2]


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


class Timer:
    """HIP events recorded on one stream around a block of launches.

    The untimed warmup is `warmup` launches and at least WARM_S of wall
    time: after host-side work (reference checks, buffer set-up) the GPU's
    clocks have dropped, and a few dozen microsecond-scale launches do not
    bring them back, so a short kernel timed right away reads up to 20% slow."""

    WARM_S = 0.03

    def __init__(self, torch, stream):
        self.torch, self.stream = torch, stream

    def run(self, fn, iters, warmup, exact_warmup=False):
        """Seconds for `iters` launches; exact_warmup=True runs exactly
        `warmup` untimed launches (the contract's W steps)."""
        torch = self.torch
        t0 = time.perf_counter()
        done = 0
        while done < warmup or (not exact_warmup and time.perf_counter() - t0 < self.WARM_S):
            with torch.cuda.stream(self.stream):
                for i in range(max(warmup, 1)):
                    fn(done + i)
            done += max(warmup, 1)
            torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        with torch.cuda.stream(self.stream):
            e0.record(self.stream)
            for i in range(iters):
                fn(warmup + i)
            e1.record(self.stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) * 1e-3  # seconds


def ring_count(bytes_per_slot):
    return max(2, int(math.ceil(RING_BYTES / bytes_per_slot)))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--no-compare", action="store_true")
    ap.add_argument("--skip-cpu", action="store_true")
    ap.add_argument("--sweep", action="store_true")
    ap.add_argument("--timeline", action="store_true",
                    help="only the per-wave phase timeline of the headline shape's variants")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU (the batched FFT shards by rows, with no exchange "
              "between GPUs); --gpus above 1 is not supported.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2603_27569_amd as sf
    from paper_2603_27569_amd import metrics, workloads

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.Stream()
    cs = stream.cuda_stream
    T = Timer(torch, stream)
    props = torch.cuda.get_device_properties(dev)
    log(f"device {props.name} {props.gcnArchName} CUs={props.multi_processor_count}")

    if args.timeline:
        print(json.dumps({"timeline": run_timeline(torch, np, sf, dev, cs)}), flush=True)
        return

    # ------------------------------------------------------------ headline
    n, b = N_HEAD, B_HEAD
    slot_bytes = n * b * 8
    K = ring_count(3 * slot_bytes)
    x0 = torch.from_numpy(workloads.plain_normal(n, b)).to(dev)
    gen = torch.Generator(device=dev)
    gen.manual_seed(1002)
    xs = [x0] + [torch.randn(n * b, dtype=torch.complex64, device=dev, generator=gen).view(b, n)
                 for _ in range(K - 1)]
    ys = [torch.empty_like(x0) for _ in range(K)]
    zs = [torch.empty_like(x0) for _ in range(K)]
    fwd = sf.Plan(n, b, sf.FFT_FORWARD)
    bwd = sf.Plan(n, b, sf.FFT_BACKWARD)
    variant = fwd.describe()["variant"]["name"]
    log(f"headline n={n} batch={b} variant={variant} ring={K} slots")

    def step(i):
        j = i % K
        fwd.exec(xs[j].data_ptr(), ys[j].data_ptr(), cs)
        bwd.exec(ys[j].data_ptr(), zs[j].data_ptr(), cs)

    # The contract's figure: exactly K timed steps after W warmup steps.
    t_step = T.run(step, args.steps, args.warmup, exact_warmup=True) / args.steps
    # Per-launch figures for the roofline: median of 5 event-timed runs.
    t_fwd = median_of(T, lambda i: fwd.exec(xs[i % K].data_ptr(), ys[i % K].data_ptr(), cs),
                      args.steps, args.warmup)
    t_bwd = median_of(T, lambda i: bwd.exec(ys[i % K].data_ptr(), zs[i % K].data_ptr(), cs),
                      args.steps, args.warmup)
    flops_step = 2 * metrics.fft_flops(n, b)
    bytes_launch = metrics.fft_bytes(n, b)
    gflops = flops_step / t_step / 1e9
    log(f"step {t_step * 1e6:.2f} us  fwd {t_fwd * 1e6:.2f} us  bwd {t_bwd * 1e6:.2f} us  "
        f"{gflops:.0f} GFLOPS")

    # accuracy of the timed path on slot 0 (forward) and its backward
    torch.cuda.synchronize()
    acc = {}
    x_h = x0.cpu().numpy()
    y_h = ys[0].cpu().numpy()
    ok, worst, med, ab = metrics.gate(y_h, ref_fft(np, x_h), x_h)
    okb, worstb, _, _ = metrics.gate(zs[0].cpu().numpy(), ref_fft(np, y_h, inverse=True), y_h)
    acc = {"reference": "numpy.fft FP64", "forward_worst_rel_rms": worst,
           "forward_median_rel_rms": med, "backward_worst_rel_rms": worstb,
           "gates_pass": bool(ok and okb)}

    # -------------------------------------------------------------- roofline
    t_kernel = (t_fwd + t_bwd) / 2
    kernel_family = "k_stockham_wx" if fwd.describe()["variant"].get("wave_exchange") else "k_stockham"
    achieved = bytes_launch / t_kernel / 1e9
    traffic = None
    try:
        with open(TRAFFIC_FILE) as f:
            tr = json.load(f)
        if tr.get("source_hash") == kernel_source_hash() and tr.get("variant") == variant:
            traffic = tr["bytes_per_launch"]
    except (OSError, ValueError, KeyError):
        pass
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "kernel": f"{kernel_family}<{variant}>", "algorithmic_bytes_per_launch": bytes_launch,
                "avg_launch_us": round(t_kernel * 1e6, 3)}

    # ----------------------------------------------------- reference kernels
    # Hand-written HIP references (libstockref.so), launched through ctypes on
    # the bench stream like the transform: an empty kernel in the headline's
    # launch shape, a copy of the same bytes in that shape (one workgroup of
    # 256 lanes per row, the transform's streaming 8-byte accesses), the same
    # bytes in a wide grid (16-byte accesses), and a large copy for the
    # device's practical HBM rate.
    from paper_2603_27569_amd import reference as ref
    refs = {}
    cp_src = [xs[j] for j in range(K)]
    cp_dst = [ys[j] for j in range(K)]
    t_empty = median_of(T, lambda i: ref.empty(b, 256, cs), args.steps, args.warmup)
    t_copy = median_of(T, lambda i: ref.copy_rows(cp_src[i % K].data_ptr(), cp_dst[i % K].data_ptr(),
                                                  n, b, 256, cs), args.steps, args.warmup)
    t_wide = median_of(T, lambda i: ref.copy_wide(cp_src[i % K].data_ptr(), cp_dst[i % K].data_ptr(),
                                                  slot_bytes, cs), args.steps, args.warmup)
    refs["empty_kernel_same_grid_us"] = round(t_empty * 1e6, 3)
    refs["copy_same_grid"] = {"us": round(t_copy * 1e6, 3),
                              "GBs": round(bytes_launch / t_copy / 1e9, 1),
                              "shape": f"{b} workgroups x 256 lanes, 8-byte streaming accesses"}
    refs["copy_wide_grid_same_bytes"] = {"us": round(t_wide * 1e6, 3),
                                         "GBs": round(bytes_launch / t_wide / 1e9, 1)}
    big = 256 << 20
    bsrc = torch.empty(big // 8, dtype=torch.complex64, device=dev)
    bdst = torch.empty_like(bsrc)
    t_big = median_of(T, lambda i: ref.copy_wide(bsrc.data_ptr(), bdst.data_ptr(), big, cs),
                      max(20, args.steps // 10), 5)
    refs["copy_wide_256MiB"] = {"us": round(t_big * 1e6, 3), "GBs": round(2 * big / t_big / 1e9, 1)}
    del bsrc, bdst
    # The LDS roof of the exchange (the secondary roof): 32 KiB written and
    # read back per round per workgroup, barrier after each half, 256 lanes.
    # One workgroup per CU (the headline's occupancy) gives the time of one
    # exchange; four per CU give the LDS's aggregate rate.
    rounds = 256
    lds = {}
    for per_cu in (1, 4):
        g = 256 * per_cu
        lout = torch.empty(g * 256, dtype=torch.float32, device=dev)
        t_l = median_of(T, lambda i: ref.lds_exchange(g, rounds, lout.data_ptr(), cs),
                        max(10, args.steps // 50), 3)
        lds[f"{per_cu}_per_cu"] = {"us_per_exchange": round(t_l / rounds * 1e6, 4),
                                   "TBs_aggregate": round(g * rounds * 65536 / t_l / 1e12, 2)}
        del lout
    refs["lds_exchange_32KiB"] = lds
    # How close the transform comes to moving its bytes with no arithmetic in
    # the same launch shape.
    roofline["frac_of_same_size_copy"] = round(t_copy / t_kernel, 4)
    roofline["copy_same_grid_us"] = round(t_copy * 1e6, 3)
    log("references", refs)

    # ------------------------------------------------------------ comparisons
    comps = {}
    if not args.no_compare:
        comps = compare(args, torch, np, sf, metrics, workloads, T, dev, cs)
    sweep = run_sweep(args, torch, sf, metrics, T, dev, cs) if args.sweep else None

    # ------------------------------------------------------------ cpu baseline
    cpu = None
    if not args.skip_cpu:
        cpu = cpu_baseline(np, x0.cpu().numpy(), flops_step, n, b)

    out = {
        "metric": "c2c FP32 FFT GFLOPS & %HBM peak, N=4096 b=256; ragged/fwd+bwd vs plain",
        "value": round(gflops, 1),
        "unit": "GFLOPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(t_step * 1e3, 6),
        "higher_is_better": True,
        "scaling": "weak",
        # The paper's own figure for this metric and workload (Table VI, on an
        # Apple M1 GPU): context for the ratio, not a like-for-like target.
        "vs_baseline": round(gflops / PAPER_CONTEXT["gflops"], 3),
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "c2c fp32 fft forward+backward, n=4096, batch=256 (complex64 rows)",
                   "n": n, "batch": b, "variant": variant, "ring_slots": K,
                   "parallelism": "single gpu"},
        "pct_hbm_peak": round(100 * 2 * bytes_launch / t_step / 1e9 / HBM_PEAK_GBS, 2),
        "forward_us": round(t_fwd * 1e6, 3),
        "backward_us": round(t_bwd * 1e6, 3),
        "accuracy": acc,
        "roofline": roofline,
        "cpu_baseline": cpu,
        "reference_kernels": refs,
        "comparisons": comps,
        "paper_context": PAPER_CONTEXT,
    }
    if sweep is not None:
        out["sweep"] = sweep
    print(json.dumps(out), flush=True)


def cpu_baseline(np, x_h, flops_step, n, b, seconds=10.0):
    """The FP64 oracle on the host cores: full steps (forward + backward of
    all rows) repeated for about `seconds`, median step time; plus one thread
    on a 16-row sample."""
    import oracle
    threads = oracle.max_threads()
    times = []
    t_begin = time.perf_counter()
    while len(times) < 3 or time.perf_counter() - t_begin < seconds:
        t0 = time.perf_counter()
        yh = oracle.fft(x_h)
        oracle.fft(yh, inverse=True)
        times.append(time.perf_counter() - t0)
    times.sort()
    tc = times[len(times) // 2]
    rows1 = 16
    oracle.set_threads(1)
    try:
        t1s = []
        for _ in range(3):
            t0 = time.perf_counter()
            yh = oracle.fft(x_h[:rows1])
            oracle.fft(yh, inverse=True)
            t1s.append(time.perf_counter() - t0)
    finally:
        oracle.set_threads(threads)
    t1 = sorted(t1s)[1] * b / rows1
    return {"value": round(flops_step / tc / 1e9, 3), "unit": "GFLOPS", "cores": threads,
            "kind": "oracle",
            "sample": f"{len(times)} full steps (forward + backward of {b} rows of N={n}) in FP64, "
                      f"median step time",
            "seconds_per_step": round(tc, 4),
            "one_thread": {"value": round(flops_step / t1 / 1e9, 3),
                           "sample": f"{rows1} rows, scaled to the step, median of 3"},
            "cpu_model": cpu_model()}


def compare(args, torch, np, sf, metrics, workloads, T, dev, cs):
    comps = {}
    iters = max(20, args.steps // 5)
    warm = max(5, args.warmup // 5)

    # Fused forward -> weight -> adjoint (N=4096, batch 512) vs the plain chain.
    n, b = 4096, 512
    x_h, w_h = workloads.spectral_energy_inputs(n, b)
    K = ring_count(2 * n * b * 8)
    from paper_2603_27569_amd import reference as ref
    x0 = torch.from_numpy(x_h).to(dev)
    w = torch.from_numpy(w_h).to(dev)
    xs = [x0] + [torch.randn(b, n, dtype=torch.complex64, device=dev) for _ in range(K - 1)]
    gs = [torch.empty_like(x0) for _ in range(K)]
    ys = [torch.empty_like(x0) for _ in range(K)]
    rows = torch.empty(b, device=dev)
    total = torch.empty(1, device=dev)
    pf = sf.Plan(n, b, sf.FFT_FORWARD, sf.FFT_ALGO_SINGLE_PASS)
    pb = sf.Plan(n, b, sf.FFT_BACKWARD, sf.FFT_ALGO_SINGLE_PASS)

    def fused(i):
        j = i % K
        sf.fft_exec_spectral_energy(pf.handle, xs[j].data_ptr(), w.data_ptr(), 0, gs[j].data_ptr(),
                                    rows.data_ptr(), total.data_ptr(), cs)

    # The unfused chain: three HIP kernels (forward, the weight step with the
    # row losses, adjoint); the fused call also writes the loss total.
    def chain(i):
        j = i % K
        pf.exec(xs[j].data_ptr(), ys[j].data_ptr(), cs)
        ref.weight_energy(ys[j].data_ptr(), w.data_ptr(), rows.data_ptr(), n, b, cs)
        pb.exec(ys[j].data_ptr(), gs[j].data_ptr(), cs)

    def launches_only(i):
        j = i % K
        pf.exec(xs[j].data_ptr(), ys[j].data_ptr(), cs)
        pb.exec(ys[j].data_ptr(), gs[j].data_ptr(), cs)

    t_fused = T.run(fused, iters, warm) / iters
    g_fused = gs[0].cpu().numpy()
    t_chain = T.run(chain, iters, warm) / iters
    g_chain = gs[0].cpu().numpy()
    t_two = T.run(launches_only, iters, warm) / iters
    w2h = 2.0 * w_h.astype(np.float64) ** 2
    ref = ref_fft(np, w2h * ref_fft(np, x_h), inverse=True)
    ok_f, rel_f, _ = metrics.grad_gate(g_fused, ref)
    ok_c, rel_c, _ = metrics.grad_gate(g_chain, ref)
    comps["fused_forward_adjoint_n4096_b512"] = {
        "fused_us": round(t_fused * 1e6, 3), "plain_chain_us": round(t_chain * 1e6, 3),
        "two_launches_us": round(t_two * 1e6, 3),
        "speedup_vs_chain": round(t_chain / t_fused, 3),
        "speedup_vs_two_launches": round(t_two / t_fused, 3),
        "fused_GBs_algorithmic": round(16 * n * b / t_fused / 1e9, 1),
        "grad_worst_row_rel_err_fused": rel_f, "grad_worst_row_rel_err_chain": rel_c,
        "equal_accuracy_gate": bool(ok_f and ok_c)}
    log("fused", comps["fused_forward_adjoint_n4096_b512"])
    del xs, gs, ys

    # Fused range compression F^-1(conj(h) F x) vs its unfused chain.
    comps["matched_filter_n4096_b256"] = compare_matched(torch, np, sf, metrics, workloads, T, dev,
                                                         cs, iters, warm)
    log("matched", comps["matched_filter_n4096_b256"])

    # Four-step vs single-pass at N=8192 / 16384, batch 1024.
    for n in (8192, 16384):
        b = 1024
        x_h, _ = workloads.chirp_noise(n, b)
        K = ring_count(2 * n * b * 8)
        xs = [torch.from_numpy(x_h).to(dev)] + [torch.randn(b, n, dtype=torch.complex64, device=dev)
                                                for _ in range(K - 1)]
        ys = [torch.empty_like(xs[0]) for _ in range(K)]
        rec = {}
        for name, algo in (("single_pass", sf.FFT_ALGO_SINGLE_PASS), ("four_step", sf.FFT_ALGO_FOUR_STEP)):
            p = sf.Plan(n, b, sf.FFT_FORWARD, algo)
            t = T.run(lambda i: p.exec(xs[i % K].data_ptr(), ys[i % K].data_ptr(), cs), iters, warm) / iters
            p.exec(xs[0].data_ptr(), ys[0].data_ptr(), cs)
            torch.cuda.synchronize()
            ok, worst, _, _ = metrics.gate(ys[0].cpu().numpy(), ref_fft(np, x_h), x_h)
            rec[name] = {"us": round(t * 1e6, 3), "GBs_algorithmic": round(16 * n * b / t / 1e9, 1),
                         "gflops": round(metrics.gflops(n, b, t), 1), "worst_rel_rms": worst,
                         "gates_pass": ok, "variant": p.describe().get("four_step", p.describe()["variant"])["name"]}
            p.close()
        comps[f"single_vs_four_step_n{n}_b{b}"] = rec
        log(f"n{n}", rec)
        del xs, ys

    # 16-bit storage (binary16 / bfloat16 pairs, FP32 arithmetic): half the
    # bytes of the FP32 path at the same transform.
    comps["storage_16bit"] = compare_lowp(torch, np, sf, metrics, workloads, T, dev, cs, iters, warm)
    log("storage_16bit", comps["storage_16bit"])

    # Lengths beyond one LDS-resident transform: the four-step only (two
    # passes over HBM, so at most half the algorithmic rate of the peak).
    for n, b in ((1 << 16, 256), (1 << 20, 16)):
        x_h = workloads.complex_normal((b, n), seed=1006 + n % 997)
        K = ring_count(2 * n * b * 8)
        xs = [torch.from_numpy(x_h).to(dev)] + [torch.randn(b, n, dtype=torch.complex64, device=dev)
                                                for _ in range(K - 1)]
        ys = [torch.empty_like(xs[0]) for _ in range(K)]
        p = sf.Plan(n, b, sf.FFT_FORWARD)
        t = T.run(lambda i: p.exec(xs[i % K].data_ptr(), ys[i % K].data_ptr(), cs), iters, warm) / iters
        p.exec(xs[0].data_ptr(), ys[0].data_ptr(), cs)
        torch.cuda.synchronize()
        rows = min(b, 4)
        ok, worst, _, _ = metrics.gate(ys[0][:rows].cpu().numpy(), ref_fft(np, x_h[:rows]), x_h[:rows])
        comps[f"four_step_n{n}_b{b}"] = {
            "us": round(t * 1e6, 3), "GBs_algorithmic": round(16 * n * b / t / 1e9, 1),
            "GBs_moved_two_passes": round(32 * n * b / t / 1e9, 1),
            "gflops": round(metrics.gflops(n, b, t), 1), "worst_rel_rms_checked_rows": worst,
            "gates_pass": bool(ok), "variant": p.describe()["four_step"]["name"]}
        log(f"four-step n{n}", comps[f"four_step_n{n}_b{b}"])
        p.close()
        del xs, ys

    # Exchange tiers at N = 4096 on one radix plan (8 8 8 8) and one twiddle
    # table: every exchange through the LDS (padded) against the exchanges
    # after passes 0 and 2 as in-wave transposes (one or two groups per lane).
    comps["exchange_tiers_n4096"] = compare_exchange_tiers(torch, np, sf, metrics, workloads, T,
                                                           dev, cs, iters, warm)
    log("exchange tiers", comps["exchange_tiers_n4096"])

    # Ragged persistent launch vs per-size plain launches.
    try:
        comps["ragged_2000"] = compare_ragged(args, torch, np, sf, metrics, workloads, T, dev, cs, iters, warm)
        log("ragged", comps["ragged_2000"])
    except sf.StockfftError as e:
        comps["ragged_2000"] = {"error": str(e)}
    return comps


EXCHANGE_TIERS = (("lds", "n4096_e8_b1_p4_r8.8.8.8_pt"),
                  ("in_wave_one_group_per_lane", "n4096_e8_b1_px_r8.8.8.8_pt_wx1"),
                  ("in_wave_two_groups_per_lane", "n4096_e16_b1_px_r8.8.8.8_pt_wx2"),
                  ("in_wave_two_members_per_lane", "n4096_e16_b1_px_r8.8.8.8_pt_wm2"))


def compare_exchange_tiers(torch, np, sf, metrics, workloads, T, dev, cs, iters, warm):
    n = 4096
    out = {}
    for b in (32, 256, 2048):
        x_h = workloads.plain_normal(n, b, seed=4242 + b)
        K = ring_count(2 * n * b * 8)
        xs = [torch.from_numpy(x_h).to(dev)] + [torch.randn(b, n, dtype=torch.complex64, device=dev)
                                                for _ in range(K - 1)]
        ys = [torch.empty_like(xs[0]) for _ in range(K)]
        want = ref_fft(np, x_h)
        rec = {}
        for label, name in EXCHANGE_TIERS:
            p = sf.Plan(n, b, sf.FFT_FORWARD, sf.FFT_ALGO_SINGLE_PASS, name)
            t = T.run(lambda i: p.exec(xs[i % K].data_ptr(), ys[i % K].data_ptr(), cs), iters, warm) / iters
            p.exec(xs[0].data_ptr(), ys[0].data_ptr(), cs)
            torch.cuda.synchronize()
            ok, worst, _, _ = metrics.gate(ys[0].cpu().numpy(), want, x_h)
            rec[label] = {"variant": name, "us": round(t * 1e6, 3),
                          "pct_hbm": round(100 * 16 * n * b / t / 1e9 / HBM_PEAK_GBS, 2),
                          "worst_rel_rms": worst, "gates_pass": bool(ok)}
            p.close()
        out[f"b{b}"] = rec
        del xs, ys
    return out


def compare_lowp(torch, np, sf, metrics, workloads, T, dev, cs, iters, warm):
    out = {}
    n = 4096
    for b in (256, 2048, 16384):
        x_h = workloads.complex_normal((b, n), seed=1007 + b)
        rec = {}
        K = ring_count(2 * n * b * 8)
        xs = [torch.from_numpy(x_h).to(dev)] + [torch.randn(b, n, dtype=torch.complex64, device=dev)
                                                for _ in range(K - 1)]
        ys = [torch.empty_like(xs[0]) for _ in range(K)]
        p = sf.Plan(n, b, sf.FFT_FORWARD, sf.FFT_ALGO_SINGLE_PASS)
        t32 = T.run(lambda i: p.exec(xs[i % K].data_ptr(), ys[i % K].data_ptr(), cs), iters, warm) / iters
        rec["fp32_us"] = round(t32 * 1e6, 3)
        del xs, ys
        for key, fmt, io, dt in (("f16", "f16", sf.FFT_IO_C16, torch.float16),
                                 ("bf16", "bf16", sf.FFT_IO_BC16, torch.bfloat16),
                                 ("f16_matrix_cores", "f16", sf.FFT_IO_C16_MMA, torch.float16),
                                 ("bf16_matrix_cores", "bf16", sf.FFT_IO_BC16_MMA, torch.bfloat16)):
            mma = key.endswith("matrix_cores")
            stored, xv = workloads.to_storage(x_h, fmt)
            t0 = torch.from_numpy(np.ascontiguousarray(stored))
            if fmt == "bf16":
                t0 = t0.view(torch.int16).view(torch.bfloat16)
            K2 = ring_count(2 * n * b * 4)
            xs = [t0.to(dev)] + [torch.randn(b, n, 2, device=dev).to(dt) for _ in range(K2 - 1)]
            ys = [torch.empty_like(xs[0]) for _ in range(K2)]
            t = T.run(lambda i: sf.fft_exec_io(p.handle, xs[i % K2].data_ptr(), ys[i % K2].data_ptr(), io, cs),
                      iters, warm) / iters
            sf.fft_exec_io(p.handle, xs[0].data_ptr(), ys[0].data_ptr(), io, cs)
            torch.cuda.synchronize()
            rows = min(b, 32)
            yh = ys[0][:rows].cpu()
            if fmt == "bf16":
                yv = workloads.bf16_value(yh.view(torch.int16).numpy().view(np.uint16)).astype(np.float64)
            else:
                yv = yh.numpy().astype(np.float64)
            ok, worst, med, _ = metrics.gate_storage(yv[..., 0] + 1j * yv[..., 1], ref_fft(np, xv[:rows]),
                                                     xv[:rows], fmt, mma=mma)
            rec[key] = {"us": round(t * 1e6, 3), "speedup_vs_fp32": round(t32 / t, 3),
                        "GBs_moved_algorithmic": round(8 * n * b / t / 1e9, 1),
                        "pct_hbm_peak": round(100 * 8 * n * b / t / 1e9 / HBM_PEAK_GBS, 2),
                        "worst_rel_rms": worst, "median_rel_rms": med,
                        "unit_roundoff": metrics.STORAGE_UNIT_ROUNDOFF[fmt], "gates_pass": bool(ok)}
            if mma:
                rec[key]["gate_factor_u"] = round(metrics.mma_gate_factor(fmt), 3)
            del xs, ys
        p.close()
        out[f"n{n}_b{b}"] = rec
    return out


def compare_matched(torch, np, sf, metrics, workloads, T, dev, cs, iters, warm):
    n, b = 4096, 256
    x_h, h_h = workloads.range_compression_inputs(n, b)
    K = ring_count(2 * n * b * 8)
    xs = [torch.from_numpy(x_h).to(dev)] + [torch.randn(b, n, dtype=torch.complex64, device=dev)
                                            for _ in range(K - 1)]
    ys = [torch.empty_like(xs[0]) for _ in range(K)]
    zs = [torch.empty_like(xs[0]) for _ in range(K)]
    from paper_2603_27569_amd import reference as ref
    h = torch.from_numpy(h_h).to(dev)
    pf = sf.Plan(n, b, sf.FFT_FORWARD, sf.FFT_ALGO_SINGLE_PASS)
    pb = sf.Plan(n, b, sf.FFT_BACKWARD, sf.FFT_ALGO_SINGLE_PASS)

    def fused(i):
        j = i % K
        sf.fft_exec_matched_filter(pf.handle, xs[j].data_ptr(), h.data_ptr(), zs[j].data_ptr(), cs)

    # The unfused chain: three HIP kernels (forward, multiply by conj(h) / n,
    # backward).
    def chain(i):
        j = i % K
        pf.exec(xs[j].data_ptr(), ys[j].data_ptr(), cs)
        ref.filter_multiply(ys[j].data_ptr(), h.data_ptr(), n, b, cs)
        pb.exec(ys[j].data_ptr(), zs[j].data_ptr(), cs)

    def two(i):
        j = i % K
        pf.exec(xs[j].data_ptr(), ys[j].data_ptr(), cs)
        pb.exec(ys[j].data_ptr(), zs[j].data_ptr(), cs)

    t_f = T.run(fused, iters, warm) / iters
    torch.cuda.synchronize()
    z_f = zs[0].cpu().numpy()
    t_c = T.run(chain, iters, warm) / iters
    torch.cuda.synchronize()
    z_c = zs[0].cpu().numpy()
    t_2 = T.run(two, iters, warm) / iters
    ref = ref_fft(np, np.conj(h_h.astype(np.complex128)) * ref_fft(np, x_h), inverse=True) / n
    ok_f, w_f, _, _ = metrics.gate(z_f, ref, x_h)
    ok_c, w_c, _, _ = metrics.gate(z_c, ref, x_h)
    pf.close()
    pb.close()
    return {"fused_us": round(t_f * 1e6, 3), "plain_chain_us": round(t_c * 1e6, 3),
            "two_launches_us": round(t_2 * 1e6, 3), "speedup_vs_chain": round(t_c / t_f, 3),
            "speedup_vs_two_launches": round(t_2 / t_f, 3),
            "fused_GBs_algorithmic": round(16 * n * b / t_f / 1e9, 1),
            "worst_rel_rms_fused": w_f, "worst_rel_rms_chain": w_c,
            "equal_accuracy_gate": bool(ok_f and ok_c)}


def compare_ragged(args, torch, np, sf, metrics, workloads, T, dev, cs, iters, warm):
    sizes, offs, data = workloads.ragged()
    total = int(sizes.sum())
    K = ring_count(2 * total * 8)
    plan = sf.RaggedPlan(sizes)
    xs = [torch.from_numpy(data).to(dev)] + [torch.randn(total, dtype=torch.complex64, device=dev)
                                             for _ in range(K - 1)]
    ys = [torch.empty_like(xs[0]) for _ in range(K)]
    # grouped copies for the per-size comparator (its best case: contiguous rows)
    order = [np.nonzero(sizes == s)[0] for s in workloads.SIZES]
    gx = []
    gy = []
    for j in range(K):
        ins = [torch.empty(len(idx) * s, dtype=torch.complex64, device=dev) if len(idx) else None
               for idx, s in zip(order, workloads.SIZES)]
        outs = [torch.empty_like(t) if t is not None else None for t in ins]
        # gather each size's rows in plan order (device copies, done once)
        for t, idx, s in zip(ins, order, workloads.SIZES):
            if t is None:
                continue
            src = xs[j]
            parts = [src[int(offs[i]):int(offs[i]) + int(s)] for i in idx]
            t.copy_(torch.cat(parts))
        gx.append(ins)
        gy.append(outs)
    t_r = T.run(lambda i: plan.exec(xs[i % K].data_ptr(), ys[i % K].data_ptr(), cs), iters, warm) / iters
    t_rd = T.run(lambda i: plan.exec_direct(xs[i % K].data_ptr(), ys[i % K].data_ptr(), cs),
                 iters, warm) / iters

    def plain(i):
        j = i % K
        plan.exec_plain([t.data_ptr() if t is not None else 0 for t in gx[j]],
                        [t.data_ptr() if t is not None else 0 for t in gy[j]], cs)

    t_p = T.run(plain, iters, warm) / iters
    # The comparator's launches captured in a graph as well (one replay per
    # step); every replay of slot 0 must equal the eager result.
    L = min(K, 16)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=T.stream):
        gcs = torch.cuda.current_stream().cuda_stream
        for j in range(L):
            plan.exec_plain([t.data_ptr() if t is not None else 0 for t in gx[j]],
                            [t.data_ptr() if t is not None else 0 for t in gy[j]], gcs)
    reps = max(2, iters // L)
    t_pg = T.run(lambda i: g.replay(), reps, 2) / (reps * L)
    torch.cuda.synchronize()
    replay_out = [t.clone() if t is not None else None for t in gy[0]]
    plain(0)
    torch.cuda.synchronize()
    graph_matches_eager = all(a is None or torch.equal(a, c) for a, c in zip(replay_out, gy[0]))
    del g
    torch.cuda.synchronize()
    plan.exec(xs[0].data_ptr(), ys[0].data_ptr(), cs)
    torch.cuda.synchronize()
    y = ys[0].cpu().numpy()
    worst = 0.0
    ok = True
    for s in workloads.SIZES:
        idx = np.nonzero(sizes == s)[0]
        xr = np.stack([data[offs[i]:offs[i] + s] for i in idx])
        yr = np.stack([y[offs[i]:offs[i] + s] for i in idx])
        g_ok, w_, _, _ = metrics.gate(yr, ref_fft(np, xr), xr)
        ok &= g_ok
        worst = max(worst, w_)
    flops = sum(metrics.fft_flops(int(s)) for s in sizes)
    return {"transforms": int(len(sizes)), "elements": total,
            "persistent_graph_us": round(t_r * 1e6, 3),
            "persistent_direct_launch_us": round(t_rd * 1e6, 3),
            "speedup_direct_launch": round(t_p / t_rd, 3),
            "per_size_plain_us": round(t_p * 1e6, 3),
            "per_size_plain_graph_us": round(t_pg * 1e6, 3),
            "plain_graph_matches_eager": bool(graph_matches_eager),
            "speedup": round(t_p / t_r, 3), "speedup_vs_plain_graph": round(t_pg / t_r, 3), "persistent_GBs_algorithmic": round(16 * total / t_r / 1e9, 1),
            "persistent_gflops": round(flops / t_r / 1e9, 1), "worst_rel_rms": worst, "gates_pass": bool(ok)}


def phase_names(passes):
    names = ["input loads"]
    for p in range(passes):
        names.append(f"pass {p + 1}")
        if p + 1 < passes:
            names.append(f"exchange {p + 1}")
    return names + ["stores issued", "stores completed"]


def run_timeline(torch, np, sf, dev, cs, reps=20):
    """Per-wave phase times of the single-pass transform at N=4096 x 256 for
    each variant the reference library stamps (libstockref.so ref_timeline):
    medians over every wave of `reps` launches on ring-rotated inputs.  Phase
    durations come from the shader clock, scaled to microseconds by its
    ratio to the 100 MHz real-time counter over each wave's life; the start
    skew and the span are taken from the real-time counter (one clock for
    the whole chip)."""
    from paper_2603_27569_amd import reference as ref
    n, b = N_HEAD, B_HEAD
    K = ring_count(2 * n * b * 8)
    gen = torch.Generator(device=dev)
    gen.manual_seed(77)
    xs = [torch.randn(b, n, dtype=torch.complex64, device=dev, generator=gen) for _ in range(K)]
    ys = [torch.empty_like(xs[0]) for _ in range(K)]
    out = {}
    by_name = {v["name"]: i for i, v in enumerate(sf.variants())}
    for name in ref.timeline_variants():
        d = sf.fft_variant_describe(by_name[name])
        waves = d["threads"] // 64
        tw = torch.from_numpy(sf.fft_variant_twiddles(by_name[name])).to(dev)
        st = torch.zeros(b * waves * 32, dtype=torch.int64, device=dev)
        rows = []
        for r in range(reps + 3):
            j = r % K
            ref.timeline(name, xs[j].data_ptr(), ys[j].data_ptr(), tw.data_ptr(), b, False,
                         st.data_ptr(), cs)
            torch.cuda.synchronize()
            if r >= 3:  # the first launches warm the code and the tables
                rows.append(st.view(b * waves, 32).cpu().numpy().copy())
        a = np.concatenate(rows).astype(np.float64)
        last = 2 * d["passes"] + 2
        rt, ct = a[:, :last + 1], a[:, 16:16 + last + 1]
        ratio = (ct[:, last] - ct[:, 0]) / ((rt[:, last] - rt[:, 0]) * 0.01)  # cycles per us
        dur = np.diff(ct, axis=1) / ratio[:, None]
        names = phase_names(d["passes"])
        per_launch = np.split(rt, reps)
        spans = [(x[:, last].max() - x[:, 0].min()) * 0.01 for x in per_launch]
        skews = [(x[:, 0].max() - x[:, 0].min()) * 0.01 for x in per_launch]
        life = (rt[:, last] - rt[:, 0]) * 0.01
        out[name] = {
            "waves_per_workgroup": waves,
            "phase_us_median": {k: round(float(np.median(dur[:, i])), 3) for i, k in enumerate(names)},
            "phase_us_p90": {k: round(float(np.percentile(dur[:, i], 90)), 3) for i, k in enumerate(names)},
            "wave_life_us_median": round(float(np.median(life)), 3),
            "start_skew_us_median": round(float(np.median(skews)), 3),
            "first_start_to_last_end_us_median": round(float(np.median(spans)), 3),
            "shader_clock_mhz_median": round(float(np.median(ratio)), 1),
        }
        log("timeline", name, out[name])
    return out


def run_sweep(args, torch, sf, metrics, T, dev, cs):
    res = {"batch_n4096": [], "size_b1024": []}
    iters = max(20, args.steps // 5)
    for b in (1, 4, 16, 64, 128, 256, 512, 1024, 2048, 4096):
        res["batch_n4096"].append(_time_plain(torch, sf, metrics, T, dev, cs, 4096, b, iters))
    for n in (256, 512, 1024, 2048, 4096, 8192, 16384):
        res["size_b1024"].append(_time_plain(torch, sf, metrics, T, dev, cs, n, 1024, iters))
    return res


def _time_plain(torch, sf, metrics, T, dev, cs, n, b, iters):
    K = ring_count(2 * n * b * 8)
    K = min(K, 4096)
    xs = [torch.randn(b, n, dtype=torch.complex64, device=dev) for _ in range(K)]
    ys = [torch.empty_like(xs[0]) for _ in range(K)]
    p = sf.Plan(n, b, sf.FFT_FORWARD)
    t = T.run(lambda i: p.exec(xs[i % K].data_ptr(), ys[i % K].data_ptr(), cs), iters, 10) / iters
    rec = {"n": n, "batch": b, "us": round(t * 1e6, 3), "gflops": round(metrics.gflops(n, b, t), 1),
           "pct_hbm": round(100 * 16 * n * b / t / 1e9 / HBM_PEAK_GBS, 2),
           "variant": p.describe()["variant"]["name"]}
    p.close()
    return rec


if __name__ == "__main__":
    main()
