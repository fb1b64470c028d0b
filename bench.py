#!/usr/bin/env python3
"""Throughput of the X-engine on one MI355X.

Workload (default ``cylinder``): the 192-input cylinder array (96 dual-pol
feeds, paper Sec. 1) with a 1024-point spectrum (Sec. 2.1), 8192 spectra per
integration, 4+4-bit seeded synthetic voltages (quantised Gaussian sigma 2.5
plus three correlated point sources), resident in HBM before timing.

One step = one pass of the plain engine over one integration, delivered
into a device buffer: xeng_correlate_dump (stage, unpack, int8 MFMA
contraction, integrate, with the epilogue writing the visibilities straight
into the caller's buffer).  The same step as separate xeng_correlate (into
the HBM accumulator) + xeng_dump (copy out) calls is timed after it and
reported as ms_per_step_separate_calls.

Printed: one JSON line with the useful complex-MAC rate of the step
(N(N+1)/2 * F * T per step, Hermitian triangle with autos), its real-time
factor at 250 MSPS real sampling (125e6 complex spectra/s per input across
all channels), the roofline of the dominant kernel (timed live with HIP
events on the engine's stream) and the CPU oracle timed on a bounded sample
of the same workload.

Other workloads (one JSON line each, same keys plus a comparison):
  --workload batch    12 arrays of uneven N, F, T (seeded): one batched
                      correlate-and-dump call (persistent launch in a captured
                      graph) per step, against 12 plain correlate-and-dump
                      calls on the same stream; both autotuned first; outputs
                      compared bit for bit.
  --workload requant  the F stage's equaliser / 4-bit requantiser at the
                      cylinder shape (PFB words [8192][1024][192] -> packed
                      bytes), HBM-bound: samples/s and GB/s against 8 TB/s.
  --workload ingest   packet ingest / corner turn: 16384 time blocks x 8
                      boards x 32 channels of the paper's 8208-byte packets,
                      shuffled with 1% loss -> the X-engine's input block
                      (HBM-bound).
  --workload chan     F-stage channeliser at the cylinder shape: 192 int8 ADC
                      streams -> 8192 spectra of 1024 channels (4-tap PFB,
                      2048-point FFT per input pair), float32.
  --workload stream   four sub-arrays (N=192/96/32/32, F=1024/1024/1024/256)
                      in two waves under a memory budget that makes the
                      second wave wait: saturating throughput of the serving
                      loop against a plain loop (one launch per block per
                      sub-array), then a paced run at the 250 MSPS block rate
                      for dump latency p50/p99.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]
       python bench.py --copy-calibration   (plain device copy of known size,
                                             for scaling HBM byte counters)
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import tempfile
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_INT8_TOPS = 5000.0      # MI355X dense int8 MFMA, 5.0 POP/s
PEAK_HBM_GBS = 8000.0        # MI355X HBM3E, 8 TB/s
OPS_PER_CMAC = 8             # 4 int8 multiplies + 4 adds per complex MAC
REALTIME_SPECTRA_PER_S = 125e6   # 250 MSPS real sampling -> 125e6 complex samples/s/input
PROFILES = os.path.join(ROOT, "profiles")
CSRC = os.path.join(ROOT, "paper_1904_07778_amd", "csrc")


def log(msg: str) -> None:
    print(msg, file=sys.stderr, flush=True)


# sources of the timed kernels (the 16-row-tile ring kernel and its
# instantiations); their counters go stale when any of them changes
KERNEL_SOURCES = ("xcorr.hpp", "xcorr16.hpp", "xcorr32.hpp", "k_x16_a.hip", "k_x16_c.hip", "k_x32_a.hip",
                  "batch.hpp", "k_batch.hip", "k_dump.hip", "xeng.hip")


# sources of the F-stage kernels, per bench workload
FSTAGE_SOURCES = {"chan": ("k_chan.hip",), "requant": ("k_requant.hip",), "ingest": ("k_ingest.hip",)}


def kernel_source_hash(names=KERNEL_SOURCES) -> str:
    """Hash of the timed kernels' source files."""
    h = hashlib.sha1()
    for name in names:
        with open(os.path.join(CSRC, name), "rb") as fh:
            h.update(name.encode() + fh.read())
    return h.hexdigest()[:16]


TUNE_FILE = os.path.join(ROOT, "paper_1904_07778_amd", "tune_gfx950.txt")
TUNE_REPS = 10   # timed calls per autotuner trial
KIND_NAMES = {0: "16-row ring", 1: "32-row ring", 2: "staging"}


def _bucket(v: int) -> int:
    """ceil(log2 v), the tuning cache's F and T buckets."""
    b = 0
    while (1 << b) < v and b < 62:
        b += 1
    return b


def tuned_choices(shapes, batched: bool) -> str:
    """The launch choices the library holds for these arrays, as text (from
    a save of the in-process tuning cache)."""
    from paper_1904_07778_amd import xeng as X
    fd, path = tempfile.mkstemp(suffix=".txt")
    os.close(fd)
    try:
        X.xeng_tune_cache_save(path)
        table = {}
        with open(path) as fh:
            for line in fh:
                f = line.split()
                if len(f) == 8 and not line.startswith("#"):
                    table[(int(f[1]), int(f[2]), int(f[3]), int(f[4]))] = (int(f[5]), int(f[6]), int(f[7]))
    finally:
        os.unlink(path)
    out = []
    for n, f, t in shapes:
        c = table.get((int(batched), n, _bucket(f), _bucket(t)))
        out.append("untuned" if c is None else
                   f"N={n}: {KIND_NAMES.get(c[0], c[0])} split {c[1]}{' own launch' if c[2] else ''}")
    plan = table.get((1, 0, 0, _bucket(len(shapes)))) if batched else None
    if plan is not None:
        out.append(f"persistent launch: {plan[1]} items per workgroup")
    return "; ".join(out)


def load_tuning(args) -> str | None:
    """Load the tuning cache (--tune-cache, else the library's shipped
    file) into the library; returns the path loaded, or None."""
    from paper_1904_07778_amd import xeng as X
    path = args.tune_cache or TUNE_FILE
    if os.path.exists(path):
        X.xeng_tune_cache_load(path)
        log(f"tuning cache loaded from {path}")
        return path
    return None


def measured_traffic(workload: str, tuned: str | None, prefix: str = "xcorr", sources=KERNEL_SOURCES):
    """HBM bytes per step from the committed rocprofv3 counter summary of this
    workload (profiles/<prefix>_<workload>_counters.txt), or None when it is
    missing, was taken on another workload, on different kernel sources or
    with other launch choices."""
    path = os.path.join(PROFILES, f"{prefix}_{workload}_counters.txt")
    try:
        with open(path) as fh:
            rec = dict(l.split(":", 1) for l in fh if ":" in l and not l.startswith("#"))
    except OSError:
        return None
    rec = {k.strip(): v.strip() for k, v in rec.items()}
    if (rec.get("workload") != workload or rec.get("kernel_source_sha1") != kernel_source_hash(sources)
            or (tuned is not None and rec.get("tuned") != tuned)):
        return None
    try:
        return float(rec["hbm_bytes_per_step"])
    except (KeyError, ValueError):
        return None


def cpu_baseline(blocks, seconds: float):
    """The oracle as it stands, on whole channels of the same input (every
    block of the integration), until about `seconds` of wall time have been
    spent."""
    import oracle
    T, F, N = blocks[0].shape
    nbl = N * (N + 1) // 2
    chunk = 16
    done, t0 = 0, time.perf_counter()
    while done < F and time.perf_counter() - t0 < seconds:
        f1 = min(F, done + chunk)
        acc = None
        for b in blocks:
            acc = oracle.accumulate(b, acc, chans=(done, f1))
        done = f1
    dt = time.perf_counter() - t0
    return {"value": nbl * done * T * len(blocks) / dt, "unit": "CMAC/s", "cores": oracle.max_threads(),
            "kind": "oracle", "host_cpu": host_cpu_model(), "build": oracle.BUILD_FLAGS,
            "sample": f"{done} of {F} channels (N={N}, {len(blocks)} x T={T}) of the same input, {dt:.1f} s"}


def copy_calibration(nbytes: int = 1 << 30, reps: int = 5) -> None:
    import torch
    x = torch.empty(nbytes, dtype=torch.uint8, device="cuda").fill_(1)
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    for _ in range(reps):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes_read": nbytes, "bytes_written": nbytes, "reps": reps}))


def hbm_probe(nbytes: int = 4 << 30, reps: int = 10) -> None:
    """Reachable HBM bandwidth on this GPU, for context beside the 8 TB/s peak:
    a device-to-device copy (read + write, 1:1) and a read-dominated
    reduction, each timed with HIP events over `reps` calls."""
    import torch
    x = torch.empty(nbytes // 8, dtype=torch.int64, device="cuda").fill_(1)
    y = torch.empty_like(x)
    stream = torch.cuda.current_stream()

    def rate(fn, moved):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return moved * reps / (e0.elapsed_time(e1) / 1e3) / 1e9

    copy = rate(lambda: y.copy_(x), 2 * nbytes)
    read = rate(lambda: torch.sum(x), nbytes)
    print(json.dumps({"hbm_probe": {"copy_read_plus_write_gbs": copy, "sum_read_gbs": read,
                                    "bytes": nbytes, "reps": reps, "peak_gbs": PEAK_HBM_GBS}}))


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--workload", default="cylinder",
                    choices=["cylinder", "dish", "dish_tiny", "batch", "stream", "requant", "ingest", "chan"])
    ap.add_argument("--stream-dumps", type=int, default=4, help="dumps per request (stream, saturating)")
    ap.add_argument("--paced-seconds", type=float, default=30.0, help="length of each paced run (stream)")
    ap.add_argument("--stream-ring", type=int, default=16, help="device ring depth in blocks per sub-array (stream)")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--settle-seconds", type=float, default=1.0,
                    help="untimed run of the step before the warm-up (plain workloads)")
    ap.add_argument("--retune", action="store_true",
                    help="autotune even where the tuning cache has a choice, and save the cache "
                         "(to --tune-cache, else the library's shipped file)")
    ap.add_argument("--tune-cache", default=None,
                    help="tuning cache to load (default: the library's shipped file); arrays it has no "
                         "choice for are autotuned")
    ap.add_argument("--batched-only", action="store_true",
                    help="batch: run warm-up + steps batched calls only (for counter runs)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true")
    ap.add_argument("--hbm-probe", action="store_true",
                    help="print the copy and read bandwidth this GPU reaches, then exit")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the X-engine shards by channel with no exchange "
              "between GPUs, and this build runs and reports a single MI355X (--gpus 1).",
              file=sys.stderr)
        return 2

    import numpy as np
    import torch

    import synth
    from paper_1904_07778_amd.xeng import Plan

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 2
    torch.cuda.set_device(0)
    # Every step runs on this one stream: inputs, outputs, the engine's
    # launches and the timing events share it, so no call waits across streams.
    torch.cuda.set_stream(torch.cuda.Stream())
    if args.copy_calibration:
        copy_calibration()
        return 0
    if args.hbm_probe:
        hbm_probe()
        return 0

    if args.workload == "batch":
        return bench_batch(args)
    if args.workload == "stream":
        return bench_stream(args)
    if args.workload == "requant":
        return bench_requant(args)
    if args.workload == "ingest":
        return bench_ingest(args)
    if args.workload == "chan":
        return bench_chan(args)

    return bench_plain(args)


def host_cpu_model() -> str:
    """Model name of the host CPU (from /proc/cpuinfo)."""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def bench_plain(args) -> int:
    """Plain engine on one workload: cylinder (default), dish or dish_tiny.

    One step = one integration: `calls` xeng_correlate calls of T samples
    (the last one fused with the dump into a device buffer:
    xeng_correlate_dump).  The plan is autotuned first, then the step runs
    for --settle-seconds (untimed, so the shader clock reaches its level
    under this load), then W warm-up and K timed steps.  Every engine call of
    the timed steps is bracketed by HIP events on the engine's stream."""
    import numpy as np
    import torch

    import synth
    from paper_1904_07778_amd.xeng import Plan

    name = args.workload
    w = synth.WORKLOADS[name]
    N, F, T, calls = w["n_inputs"], w["n_chans"], w["n_time"], w["calls"]
    nbl = N * (N + 1) // 2
    log(f"generating {name}: N={N} F={F} T={T} x {calls} calls ({calls * T * F * N / 1e9:.2f} GB)")
    t0 = time.perf_counter()
    v_host = [synth.voltages(w["recipe"], w["seed"], N, F, T, block=b) if calls > 1 else
              synth.voltages(w["recipe"], w["seed"], N, F, T) for b in range(calls)]
    log(f"generated in {time.perf_counter() - t0:.1f} s")
    v = [torch.from_numpy(h).cuda() for h in v_host]

    from paper_1904_07778_amd import xeng as X
    load_tuning(args)
    stream = torch.cuda.current_stream()
    plan = Plan([(N, F, T)], stream=stream)
    out = plan.new_output(0)
    torch.cuda.synchronize()
    tuned_ms = None
    if args.retune or "untuned" in tuned_choices([(N, F, T)], False):
        t_settle = time.perf_counter()
        while time.perf_counter() - t_settle < args.settle_seconds:
            for _ in range(8):
                plan.correlate_dump([v[0]], out=[out])
            torch.cuda.synchronize()
        tuned_ms = plan.autotune([v[0]], reps=TUNE_REPS)
        log(f"autotuned: {tuned_ms:.4f} ms per call")
        if args.retune:
            X.xeng_tune_cache_save(args.tune_cache or TUNE_FILE)
    tuned = tuned_choices([(N, F, T)], False)
    log(f"launch choice: {tuned} ({'autotuned' if tuned_ms is not None else 'tuning cache'})")

    def step(events=None):
        for k in range(calls):
            if events is not None:
                events[k][0].record(stream)
            if k + 1 < calls:
                plan.correlate([v[k]])
            else:
                plan.correlate_dump([v[k]], out=[out])
            if events is not None:
                events[k][1].record(stream)

    t_settle = time.perf_counter()
    n_settle = 0
    while time.perf_counter() - t_settle < args.settle_seconds:
        step()
        n_settle += 1
        if n_settle % 8 == 0:
            torch.cuda.synchronize()
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    log(f"settled ({n_settle} steps in {time.perf_counter() - t_settle:.1f} s), warmup {args.warmup} done")

    # Timed region: K steps back to back, bracketed by one pair of HIP events
    # on the engine's stream (an event pair around every call adds a few
    # microseconds of device time per event to the interval it measures).
    e_start, e_end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    e_start.record(stream)
    for k in range(args.steps):
        step()
    e_end.record(stream)
    torch.cuda.synchronize()
    t_total = time.perf_counter() - t_start
    dev_mean = e_start.elapsed_time(e_end) / args.steps      # device ms per step, launch gaps included
    log(f"timed {args.steps} steps in {t_total:.3f} s ({dev_mean:.4f} ms per step on the device)")
    # Spread: the same steps again with an event pair around every engine call
    ev = [[[torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)] for _ in range(calls)]
          for _ in range(args.steps)]
    torch.cuda.synchronize()
    for k in range(args.steps):
        step(ev[k])
    torch.cuda.synchronize()
    call_ms = np.array([[a.elapsed_time(b) for a, b in e] for e in ev])   # [steps][calls]
    step_dev_ms = call_ms.sum(axis=1)

    ms_separate = None
    if calls == 1:
        torch.cuda.synchronize()
        t_sep = time.perf_counter()
        for k in range(args.steps):
            plan.correlate([v[0]])
            plan.dump(0, out=[out])
        torch.cuda.synchronize()
        ms_separate = 1e3 * (time.perf_counter() - t_sep) / args.steps
        log(f"separate correlate + dump: {ms_separate:.4f} ms per step")

    ms_per_step = 1e3 * t_total / args.steps
    cmac_per_step = nbl * F * T * calls
    value = cmac_per_step / (ms_per_step / 1e3)
    in_bytes, out_bytes = calls * T * F * N, F * nbl * 8
    alg_bytes = in_bytes + out_bytes
    hbm_bound = 4 * (N + 1) < PEAK_INT8_TOPS / PEAK_HBM_GBS * 1e3
    if hbm_bound:
        achieved = alg_bytes / (dev_mean / 1e3) / 1e9
        roof = {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": achieved / PEAK_HBM_GBS}
    else:
        achieved = cmac_per_step * OPS_PER_CMAC / (dev_mean / 1e3) / 1e12
        roof = {"bound": "mfma", "achieved": achieved, "peak": PEAK_INT8_TOPS, "unit": "TOP/s",
                "frac": achieved / PEAK_INT8_TOPS}
    roof.update({"traffic": measured_traffic(name, tuned), "algorithmic_bytes": alg_bytes,
                 "hbm_gbs_algorithmic": alg_bytes / (dev_mean / 1e3) / 1e9,
                 "int8_tops": cmac_per_step * OPS_PER_CMAC / (dev_mean / 1e3) / 1e12,
                 "time": "device time of the K timed steps (one HIP event pair on the engine stream) / K"})

    cpu = None
    if not args.no_cpu_baseline:
        log("timing the CPU oracle")
        cpu = cpu_baseline(v_host, args.cpu_seconds)

    rec = {
        "metric": "X-engine complex MAC/s (Hermitian triangle incl. autos), int8-MFMA fraction at "
                  "N=192 and real-time factor",
        "value": value,
        "unit": "CMAC/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int8",
        "data": "synthetic",
        "config": {"workload": f"{name}: N={N} inputs, F={F} channels, {calls} x T={T} samples per "
                               "integration, 4+4-bit complex",
                   "n_inputs": N, "n_chans": F, "n_time": T, "calls_per_integration": calls,
                   "step": ("correlate + dump in one call (xeng_correlate_dump)" if calls == 1 else
                            f"{calls - 1} xeng_correlate calls, then xeng_correlate_dump"),
                   "settle_s": args.settle_seconds, "launch": tuned,
                   "launch_from": "autotune" if tuned_ms is not None else "tuning cache",
                   "autotuned_ms_per_call": tuned_ms},
        "kernel_ms": dev_mean,
        "step_event_ms": {"median": float(np.median(step_dev_ms)), "min": float(step_dev_ms.min()),
                          "mean": float(step_dev_ms.mean()), "max": float(step_dev_ms.max()),
                          "note": "a second pass of K steps with an event pair around every engine call"},
        "int8_mfma_frac_of_step": value * OPS_PER_CMAC / (PEAK_INT8_TOPS * 1e12),
        "rtf": value / (nbl * REALTIME_SPECTRA_PER_S),
        "rtf_full_matrix_reading": value / (nbl * REALTIME_SPECTRA_PER_S) / 2,
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    if ms_separate is not None:
        rec["ms_per_step_separate_calls"] = ms_separate
    print(json.dumps(rec), flush=True)
    plan.close()
    return 0


def _base_record(args, metric, value, ms_per_step, config):
    return {"metric": metric, "value": value, "unit": "CMAC/s", "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "int8", "data": "synthetic",
            "config": config}


def bench_batch(args) -> int:
    """Batched workload: one batched call vs 12 plain calls per step."""
    import numpy as np
    import torch

    import synth
    from paper_1904_07778_amd.xeng import Plan

    specs = synth.batch_arrays()
    shapes = [(s["n_inputs"], s["n_chans"], s["n_time"]) for s in specs]
    log(f"batch workload: {shapes}")
    dev = [torch.from_numpy(synth.voltages("noise", 4, n, f, t, array=k)).cuda()
           for k, (n, f, t) in enumerate(shapes)]
    cmac = sum(n * (n + 1) // 2 * f * t for n, f, t in shapes)
    in_bytes = sum(n * f * t for n, f, t in shapes)
    out_bytes = sum(n * (n + 1) // 2 * f * 8 for n, f, t in shapes)
    from paper_1904_07778_amd import xeng as X
    stream = torch.cuda.current_stream()
    load_tuning(args)                                    # plans start from the cached choices
    batched = Plan(shapes, stream=stream)
    plain = [Plan([sh], stream=stream) for sh in shapes]
    torch.cuda.synchronize()
    tb = tp = None
    cached = not (args.retune or "untuned" in tuned_choices(shapes, True)
                  or "untuned" in tuned_choices(shapes, False))
    if not cached:
        # the shader clock settles before the trials, and each trial times
        # enough calls that run-to-run noise does not decide the pick
        out_b0 = [batched.new_output(k) for k in range(len(shapes))]
        t_settle = time.perf_counter()
        while time.perf_counter() - t_settle < args.settle_seconds:
            for _ in range(8):
                batched.correlate_dump(dev, out=out_b0)
            torch.cuda.synchronize()
        del out_b0
        log("autotuning")
        tb = batched.autotune(dev, reps=TUNE_REPS)
        tp = sum(p.autotune([v], reps=TUNE_REPS) for p, v in zip(plain, dev))
        log(f"autotuned: batched {tb:.3f} ms, plain sum {tp:.3f} ms")
        if args.retune:
            X.xeng_tune_cache_save(args.tune_cache or TUNE_FILE)
    tuned = tuned_choices(shapes, True)
    log(f"batched launch choices: {tuned}")
    out_b = [batched.new_output(k) for k in range(len(shapes))]
    out_p = [p.new_output(0) for p in plain]
    if args.batched_only:      # counter runs: the batched steps alone
        for _ in range(args.warmup + args.steps):
            batched.correlate_dump(dev, out=out_b)
        torch.cuda.synchronize()
        log(f"ran {args.warmup + args.steps} batched steps")
        return 0

    # both forms integrate and dump in one call per plan (xeng_correlate_dump)
    def step_batched():
        batched.correlate_dump(dev, out=out_b)

    def step_plain():
        for p, v, o in zip(plain, dev, out_p):
            p.correlate_dump([v], out=[o])

    def timed(step):
        for _ in range(args.warmup):
            step()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        e0.record(stream)
        for _ in range(args.steps):
            step()
        e1.record(stream)
        torch.cuda.synchronize()
        return 1e3 * (time.perf_counter() - t0) / args.steps, e0.elapsed_time(e1) / args.steps

    ms_b, dev_ms_b = timed(step_batched)
    ms_p, dev_ms_p = timed(step_plain)
    same = all(torch.equal(a, b) for a, b in zip(out_b, out_p))
    log(f"batched {ms_b:.3f} ms/step, plain {ms_p:.3f} ms/step, identical={same}")
    rec = _base_record(args, "X-engine complex MAC/s, 12 arrays in one batched call (correlate + dump)",
                       cmac / (ms_b / 1e3), ms_b,
                       {"workload": "batch: 12 arrays, N in {16..192}, F in {256, 512, 1024}, "
                                    "T in {2048, 4096, 8192} (seed 4), 4+4-bit complex",
                        "arrays": shapes,
                        "step": "batched correlate + dump of all arrays in one call (xeng_correlate_dump)",
                        "launch": tuned, "launch_from": "tuning cache" if cached else "autotune"})
    # the mix's combined bound: its bytes at 8 TB/s or its int8 work at 5 POP/s
    t_hbm = (in_bytes + out_bytes) / (PEAK_HBM_GBS * 1e9)
    t_mfma = cmac * OPS_PER_CMAC / (PEAK_INT8_TOPS * 1e12)
    hbm_dom = t_hbm >= t_mfma
    achieved = ((in_bytes + out_bytes) / (dev_ms_b / 1e3) / 1e9 if hbm_dom
                else cmac * OPS_PER_CMAC / (dev_ms_b / 1e3) / 1e12)
    peak = PEAK_HBM_GBS if hbm_dom else PEAK_INT8_TOPS
    rec.update({
        "plain_value": cmac / (ms_p / 1e3), "plain_ms_per_step": ms_p,
        "speedup_vs_plain": ms_p / ms_b, "identical_to_plain": same,
        "device_ms_per_step": dev_ms_b, "plain_device_ms_per_step": dev_ms_p,
        "device_speedup_vs_plain": dev_ms_p / dev_ms_b,
        "autotuned_ms": {"batched": tb, "plain_sum": tp, "from_cache": cached},
        "int8_mfma_frac_of_step": cmac * OPS_PER_CMAC / (ms_b / 1e3) / (PEAK_INT8_TOPS * 1e12),
        "roofline": {"bound": "hbm" if hbm_dom else "mfma", "achieved": achieved, "peak": peak,
                     "unit": "GB/s" if hbm_dom else "TOP/s", "frac": achieved / peak,
                     "traffic": measured_traffic("batch", tuned), "algorithmic_bytes": in_bytes + out_bytes,
                     "combined_bound_ms": max(t_hbm, t_mfma) * 1e3,
                     "note": "whole step (the graph: batch kernel, any own launches, carry-over copies) "
                             "on the engine stream, against the mix's bytes at 8 TB/s or its int8 work "
                             "at 5 POP/s, whichever is longer"},
        "cpu_baseline": None,
    })
    print(json.dumps(rec), flush=True)
    batched.close()
    for p in plain:
        p.close()
    return 0 if same else 1


def bench_stream(args) -> int:
    """Streaming workload: the serving loop, with blocks pre-staged in device
    rings and with blocks copied in from pinned host rings (H2D-inclusive),
    saturating and paced, against plain per-block launches."""
    import numpy as np
    import torch

    import synth
    from paper_1904_07778_amd.serve import (BLOCK_T, Feed, HostFeed, Request, Server, drive, latency_stats,
                                            realtime_period)
    from paper_1904_07778_amd.xeng import Plan

    subs = synth.stream_subarrays()
    ring_blocks = args.stream_ring
    log(f"stream workload: {subs}")
    hosts, rings = {}, {}
    for k, s in enumerate(subs):
        n, f = s["n_inputs"], s["n_chans"]
        h = synth.voltages("sources", 5, n, f, ring_blocks * BLOCK_T, array=k, n_src=1)
        hosts[(n, f)] = torch.from_numpy(h).pin_memory()
        rings[(n, f)] = hosts[(n, f)].cuda()
    copy_stream = torch.cuda.Stream()

    def requests(n_dumps_of, waves=2):
        reqs = []
        for w in range(waves):
            for s in subs:
                reqs.append(Request(f"{s['n_inputs']}x{s['n_chans']}#{w}", s["n_inputs"], s["n_chans"],
                                    s["dump_len"], n_dumps_of(s), ring_blocks=ring_blocks))
        return reqs

    def feeds_for(reqs, h2d):
        out = {}
        for r in reqs:
            key, nb = (r.n_inputs, r.n_chans), r.n_dumps * r.dump_len // BLOCK_T
            if h2d:   # each request copies into a device ring of its own
                out[r.name] = HostFeed(hosts[key], torch.empty_like(rings[key]), nb, copy_stream)
            else:     # pre-staged: requests of one shape read the same device ring
                out[r.name] = Feed(rings[key], nb)
        return out

    fps = [r.footprint() for r in requests(lambda s: 1, waves=1)]
    budget = sum(fps)            # one wave fits; the second waits for memory
    real_need = sum(s["n_inputs"] * (s["n_inputs"] + 1) // 2 * REALTIME_SPECTRA_PER_S for s in subs)
    reqs = requests(lambda s: args.stream_dumps)
    cmac = sum(r.n_inputs * (r.n_inputs + 1) // 2 * r.n_chans * r.n_dumps * r.dump_len for r in reqs)
    in_bytes = sum(r.n_inputs * r.n_chans * r.n_dumps * r.dump_len for r in reqs)

    def saturating(h2d):
        warm = requests(lambda s: 1)
        drive(Server(budget, keep_results=False), [(0.0, r) for r in warm], feeds_for(warm, h2d),
              paced=False)                                   # warm-up (graphs, allocator)
        rq = requests(lambda s: args.stream_dumps)
        srv = Server(budget, keep_results=False)
        t = drive(srv, [(0.0, r) for r in rq], feeds_for(rq, h2d), paced=False, time_limit=600)
        srv.close()
        log(f"serving loop ({'h2d' if h2d else 'pre-staged'}): {t:.3f} s for {cmac:.3e} CMAC, "
            f"{srv.iterations} engine calls, {latency_stats(srv.done)}")
        return t, srv

    t_serve, srv = saturating(False)
    t_serve_h2d, srv_h2d = saturating(True)

    # saturating: plain loop, one launch per block per sub-array, round robin
    stream = torch.cuda.current_stream()
    t0 = time.perf_counter()
    for _wave in range(2):
        active = []
        for s in subs:
            p = Plan([(s["n_inputs"], s["n_chans"], BLOCK_T)], stream=stream)
            out = p.new_output(0)
            active.append({"s": s, "plan": p, "done": 0, "out": out,
                           "host": torch.empty(out.shape, dtype=out.dtype, pin_memory=True),
                           "blocks": args.stream_dumps * s["dump_len"] // BLOCK_T})
        while active:
            for a in list(active):
                s, p = a["s"], a["plan"]
                ring = rings[(s["n_inputs"], s["n_chans"])]
                row = (a["done"] % ring_blocks) * BLOCK_T
                p.correlate([ring[row: row + BLOCK_T]])
                a["done"] += 1
                if a["done"] * BLOCK_T % s["dump_len"] == 0:
                    p.dump(0, out=[a["out"]])
                    a["host"].copy_(a["out"], non_blocking=True)
                if a["done"] == a["blocks"]:
                    torch.cuda.synchronize()
                    p.close()
                    active.remove(a)
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t0
    log(f"plain loop: {t_plain:.3f} s")

    # paced: blocks at the real-time rate, latency of every dump
    def paced_dumps(s):
        return max(1, int(round(args.paced_seconds / (s["dump_len"] / BLOCK_T * realtime_period(s["n_chans"])))))

    def paced(h2d):
        preqs = requests(paced_dumps, waves=1)
        psrv = Server(budget, keep_results=False)
        t = drive(psrv, [(0.0, r) for r in preqs], feeds_for(preqs, h2d), paced=True,
                  time_limit=4 * args.paced_seconds + 60)
        psrv.close()
        lat = latency_stats(psrv.done)
        per = {r.name: latency_stats([d for d in psrv.done if d.name == r.name]) for r in preqs}
        log(f"paced ({'h2d' if h2d else 'pre-staged'}): {t:.2f} s, {lat}")
        return {"seconds": t, **lat, "per_subarray": per}

    paced_pre = paced(False)
    paced_h2d = paced(True)

    value = cmac / t_serve
    rec = _base_record(args, "X-engine complex MAC/s of the streaming serving loop (saturating)",
                       value, 1e3 * t_serve / max(1, srv.iterations),
                       {"workload": "stream: sub-arrays N/F = 192/1024, 96/1024, 32/1024, 32/256, "
                                    "blocks of 1024 samples, dump lengths "
                                    + "/".join(str(s["dump_len"]) for s in subs)
                                    + f", two waves of {args.stream_dumps} dumps each under a "
                                      f"budget that fits one wave; blocks pre-staged in HBM rings of {ring_blocks}",
                        "budget_bytes": budget, "ring_blocks": ring_blocks})
    rec["steps"] = srv.iterations
    rec.update({
        "plain_value": cmac / t_plain, "speedup_vs_plain": t_plain / t_serve,
        "rtf": value / real_need,
        "saturating_latency": latency_stats(srv.done),
        "h2d": {"value": cmac / t_serve_h2d, "unit": "CMAC/s", "rtf": cmac / t_serve_h2d / real_need,
                "seconds": t_serve_h2d, "engine_calls": srv_h2d.iterations,
                "h2d_gbs": in_bytes / t_serve_h2d / 1e9,
                "saturating_latency": latency_stats(srv_h2d.done),
                "note": "blocks copied from pinned host rings into per-request device rings on a copy "
                        "stream, ordered by events against the engine calls"},
        "paced": paced_pre,
        "paced_h2d": paced_h2d,
        "roofline": None, "cpu_baseline": None,
    })
    print(json.dumps(rec), flush=True)
    return 0


def bench_chan(args) -> int:
    """F-stage channeliser at the cylinder shape."""
    import torch

    from paper_1904_07778_amd.xeng import channelise

    N, F, S = 192, 1024, 8192
    n_samples = 2 * F * (S + 3)
    log(f"chan workload: {N} streams x {n_samples} samples -> [{S}][{F}][{N}] complex64")
    g = torch.Generator(device="cuda").manual_seed(13)
    adc = (torch.randn((N, n_samples), device="cuda", generator=g) * 20).round().clamp(-128, 127).to(torch.int8)
    out = torch.empty((S, F, N), dtype=torch.complex64, device="cuda")
    tables = torch.empty(4 * 2 * F + 2 * F, dtype=torch.float32, device="cuda")
    stream = torch.cuda.Stream()
    torch.cuda.synchronize()
    for _ in range(args.warmup):
        channelise(adc, F, out=out, tables=tables, stream=stream)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    for _ in range(args.steps):
        channelise(adc, F, out=out, tables=tables, stream=stream)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = 1e3 * (time.perf_counter() - t0) / args.steps
    kms = e0.elapsed_time(e1) / args.steps
    nbytes = adc.numel() + out.numel() * 8
    flops = (N // 2) * S * (5 * 2 * F * 11 + 8 * 2 * 2 * F)   # FFT + 4-tap FIR on two streams
    rec = _base_record(args, "F-stage channeliser input samples/s (cylinder shape, 1024 channels)",
                       adc.numel() / (ms / 1e3), ms,
                       {"workload": f"chan: {N} int8 streams, {S} spectra of {F} channels, 4-tap PFB, "
                                    "two real inputs per complex FFT", "n_inputs": N, "n_chans": F, "spectra": S})
    rec.update({"unit": "samples/s", "dtype": "f32", "kernel_ms": kms,
                "roofline": {"bound": "hbm", "achieved": nbytes / (kms / 1e3) / 1e9, "peak": PEAK_HBM_GBS,
                             "unit": "GB/s", "frac": nbytes / (kms / 1e3) / 1e9 / PEAK_HBM_GBS,
                             "traffic": measured_traffic("chan", None, "fstage", FSTAGE_SOURCES["chan"]),
                             "algorithmic_bytes": nbytes,
                             "fp32_tflops": flops / (kms / 1e3) / 1e12},
                "cpu_baseline": None})
    print(json.dumps(rec), flush=True)
    return 0


def bench_ingest(args) -> int:
    """Packet ingest and corner turn at the paper's packet size."""
    import numpy as np
    import torch

    from paper_1904_07778_amd.xeng import ingest

    blocks, boards, chans = 16384, 8, 32
    pay = 8 * chans * 32
    stride = 8 + pay
    n = blocks * boards
    log(f"ingest workload: {n} packets of {stride} bytes ({n * stride / 1e9:.2f} GB)")
    g = torch.Generator(device="cuda").manual_seed(11)
    order = torch.randperm(n, device="cuda", generator=g)[: n - n // 100]   # shuffled, 1% lost
    pk = torch.randint(0, 256, (order.numel(), stride), dtype=torch.uint8, device="cuda", generator=g)
    m = (order // boards).to(torch.int64) + 1000
    b = (order % boards).to(torch.int64)
    for k in range(6):
        pk[:, k] = ((m >> (8 * (5 - k))) & 0xFF).to(torch.uint8)
    pk[:, 6] = b.to(torch.uint8)
    pk[:, 7] = 3
    out = torch.empty((8 * blocks, chans, 32 * boards), dtype=torch.uint8, device="cuda")
    stream = torch.cuda.Stream()
    torch.cuda.synchronize()
    for _ in range(args.warmup):
        ingest(pk, 1000, blocks, boards, chans, 3, out=out, stream=stream)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    for _ in range(args.steps):
        ingest(pk, 1000, blocks, boards, chans, 3, out=out, stream=stream)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = 1e3 * (time.perf_counter() - t0) / args.steps
    kms = e0.elapsed_time(e1) / args.steps
    nbytes = order.numel() * stride + out.numel()           # packets read once, block written once
    rec = _base_record(args, "packet ingest / corner turn bytes/s (8208-byte packets -> X-engine block)",
                       nbytes / (ms / 1e3), ms,
                       {"workload": f"ingest: {blocks} time blocks x {boards} boards x {chans} channels, "
                                    "shuffled, 1% lost", "packets": int(order.numel())})
    rec.update({"unit": "B/s", "dtype": "u8", "kernel_ms": kms,
                "roofline": {"bound": "hbm", "achieved": nbytes / (kms / 1e3) / 1e9, "peak": PEAK_HBM_GBS,
                             "unit": "GB/s", "frac": nbytes / (kms / 1e3) / 1e9 / PEAK_HBM_GBS,
                             "traffic": measured_traffic("ingest", None, "fstage", FSTAGE_SOURCES["ingest"]),
                             "algorithmic_bytes": nbytes},
                "cpu_baseline": None})
    print(json.dumps(rec), flush=True)
    return 0


def bench_requant(args) -> int:
    """Equaliser / 4-bit requantiser at the cylinder shape."""
    import numpy as np
    import torch

    import synth
    from paper_1904_07778_amd.xeng import requantize

    T, F, N = 8192, 1024, 192
    log(f"requant workload: words [{T}][{F}][{N}] ({T * F * N * 8 / 1e9:.1f} GB)")
    gen = torch.Generator(device="cuda").manual_seed(5)
    z = torch.randn((T, F, N, 2), device="cuda", generator=gen) * 2.0**14
    v = z.round().clamp(-(2**17), 2**17 - 1).to(torch.int64) & 0x3FFFF
    del z
    words = (v[..., 0] << 18) | v[..., 1]
    del v
    gains_h = synth.eq_gains(5, N, F)
    gains = torch.from_numpy(gains_h.view(np.int32)).cuda()
    out = torch.empty((T, F, N), dtype=torch.uint8, device="cuda")
    stream = torch.cuda.Stream()
    torch.cuda.synchronize()
    with torch.cuda.stream(stream):
        for _ in range(args.warmup):
            requantize(words, gains, out=out, stream=stream)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    for _ in range(args.steps):
        requantize(words, gains, out=out, stream=stream)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = 1e3 * (time.perf_counter() - t0) / args.steps
    kms = e0.elapsed_time(e1) / args.steps
    n = T * F * N
    nbytes = n * 9 + F * N * 4
    cpu = None
    if not args.no_cpu_baseline:
        from oracle import requant as R
        rows = 0
        c0 = time.perf_counter()
        while rows < T and time.perf_counter() - c0 < args.cpu_seconds:
            R.requantize(words[rows:rows + 8].cpu().numpy().view(np.uint64), gains_h)
            rows += 8
        dt = time.perf_counter() - c0
        cpu = {"value": rows * F * N / dt, "unit": "samples/s", "cores": 1, "kind": "oracle",
               "sample": f"{rows} of {T} time rows (F={F}, N={N}), {dt:.1f} s, numpy"}
    rec = _base_record(args, "equaliser / 4-bit requantiser complex samples/s (F stage, cylinder shape)",
                       n / (ms / 1e3), ms,
                       {"workload": f"requant: PFB words [{T}][{F}][{N}] fix_18_17, gains fix_18_7 -> packed 4+4-bit",
                        "n_time": T, "n_chans": F, "n_inputs": N})
    rec.update({"unit": "samples/s", "dtype": "int32", "kernel_ms": kms,
                "roofline": {"bound": "hbm", "achieved": nbytes / (kms / 1e3) / 1e9, "peak": PEAK_HBM_GBS,
                             "unit": "GB/s", "frac": nbytes / (kms / 1e3) / 1e9 / PEAK_HBM_GBS,
                             "traffic": measured_traffic("requant", None, "fstage", FSTAGE_SOURCES["requant"]),
                             "algorithmic_bytes": nbytes},
                "cpu_baseline": cpu})
    print(json.dumps(rec), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
