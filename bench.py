#!/usr/bin/env python3
"""Throughput of the X-engine on one MI355X.

Workload (default ``cylinder``): the 192-input cylinder array (96 dual-pol
feeds, paper Sec. 1) with a 1024-point spectrum (Sec. 2.1), 8192 spectra per
integration, 4+4-bit seeded synthetic voltages (quantised Gaussian sigma 2.5
plus three correlated point sources), resident in HBM before timing.

One step = one pass of the plain engine over one integration:
xeng_correlate (stage, unpack, int8 MFMA contraction, integrate into the
HBM accumulator) + xeng_dump to a device buffer (copy out, clear).

Printed: one JSON line with the useful complex-MAC rate of the step
(N(N+1)/2 * F * T per step, Hermitian triangle with autos), its real-time
factor at 250 MSPS real sampling (125e6 complex spectra/s per input across
all channels), the roofline of the dominant kernel (timed live with HIP
events on the engine's stream) and the CPU oracle timed on a bounded sample
of the same workload.

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
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_INT8_TOPS = 5000.0      # MI355X dense int8 MFMA, 5.0 POP/s
PEAK_HBM_GBS = 8000.0        # MI355X HBM3E, 8 TB/s
OPS_PER_CMAC = 8             # 4 int8 multiplies + 4 adds per complex MAC
REALTIME_SPECTRA_PER_S = 125e6   # 250 MSPS real sampling -> 125e6 complex samples/s/input
COUNTERS_FILE = os.path.join(ROOT, "profiles", "xcorr_cylinder_counters.txt")
CSRC = os.path.join(ROOT, "paper_1904_07778_amd", "csrc")


def log(msg: str) -> None:
    print(msg, file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    """Hash of every kernel source file (the counters go stale when it changes)."""
    h = hashlib.sha1()
    for name in sorted(os.listdir(CSRC)):
        if name.endswith((".hpp", ".hip")):
            with open(os.path.join(CSRC, name), "rb") as fh:
                h.update(name.encode() + fh.read())
    return h.hexdigest()[:16]


def measured_traffic():
    """HBM bytes per launch from the committed rocprofv3 counter summary, or
    None when it is missing or was taken on a different kernel source."""
    try:
        with open(COUNTERS_FILE) as fh:
            rec = dict(l.split(":", 1) for l in fh if ":" in l and not l.startswith("#"))
    except OSError:
        return None
    rec = {k.strip(): v.strip() for k, v in rec.items()}
    if rec.get("kernel_source_sha1") != kernel_source_hash():
        return None
    try:
        return float(rec["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def cpu_baseline(v, seconds: float):
    """The oracle as it stands, on whole channels of the same input, until
    about `seconds` of wall time have been spent."""
    import oracle
    T, F, N = v.shape
    nbl = N * (N + 1) // 2
    chunk = 16
    done, t0 = 0, time.perf_counter()
    while done < F and time.perf_counter() - t0 < seconds:
        f1 = min(F, done + chunk)
        oracle.accumulate(v, chans=(done, f1))
        done = f1
    dt = time.perf_counter() - t0
    return {"value": nbl * done * T / dt, "unit": "CMAC/s", "cores": oracle.max_threads(),
            "kind": "oracle",
            "sample": f"{done} of {F} channels (N={N}, T={T}) of the same input, {dt:.1f} s"}


def copy_calibration(nbytes: int = 1 << 30, reps: int = 5) -> None:
    import torch
    x = torch.empty(nbytes, dtype=torch.uint8, device="cuda").fill_(1)
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    for _ in range(reps):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes_read": nbytes, "bytes_written": nbytes, "reps": reps}))


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="cylinder", choices=["cylinder", "dish", "dish_tiny"])
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true")
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
    if args.copy_calibration:
        copy_calibration()
        return 0

    w = synth.WORKLOADS[args.workload]
    N, F, T = w["n_inputs"], w["n_chans"], w["n_time"]
    nbl = N * (N + 1) // 2
    log(f"generating {args.workload}: N={N} F={F} T={T} ({T * F * N / 1e9:.2f} GB)")
    t0 = time.perf_counter()
    v_host = synth.voltages(w["recipe"], w["seed"], N, F, T)
    log(f"generated in {time.perf_counter() - t0:.1f} s")
    v = torch.from_numpy(v_host).cuda()

    stream = torch.cuda.Stream()
    plan = Plan([(N, F, T)], stream=stream)
    out = plan.new_output(0)
    torch.cuda.synchronize()

    for _ in range(args.warmup):
        plan.correlate([v])
        plan.dump(0, out=[out])
    torch.cuda.synchronize()
    log(f"warmup {args.warmup} done")

    ev0 = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    ev1 = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for k in range(args.steps):
        ev0[k].record(stream)
        plan.correlate([v])
        ev1[k].record(stream)
        plan.dump(0, out=[out])
    torch.cuda.synchronize()
    t_total = time.perf_counter() - t_start
    log(f"timed {args.steps} steps in {t_total:.3f} s")
    kernel_ms = float(np.mean([a.elapsed_time(b) for a, b in zip(ev0, ev1)]))

    ms_per_step = 1e3 * t_total / args.steps
    cmac_per_step = nbl * F * T
    value = cmac_per_step / (ms_per_step / 1e3)
    achieved_tops = cmac_per_step * OPS_PER_CMAC / (kernel_ms / 1e3) / 1e12
    in_bytes, out_bytes = T * F * N, F * nbl * 8
    traffic = measured_traffic()

    cpu = None
    if not args.no_cpu_baseline:
        log("timing the CPU oracle")
        cpu = cpu_baseline(v_host, args.cpu_seconds)

    rec = {
        "metric": "X-engine complex MAC/s at N=192 (Hermitian triangle incl. autos), "
                  "int8-MFMA fraction and real-time factor",
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
        "config": {"workload": f"{args.workload}: N={N} inputs, F={F} channels, "
                               f"T={T} samples per integration, 4+4-bit complex",
                   "n_inputs": N, "n_chans": F, "n_time": T, "step": "correlate + dump"},
        "int8_mfma_frac_of_step": value * OPS_PER_CMAC / (PEAK_INT8_TOPS * 1e12),
        "rtf": value / (nbl * REALTIME_SPECTRA_PER_S),
        "rtf_full_matrix_reading": value / (nbl * REALTIME_SPECTRA_PER_S) / 2,
        "kernel_ms": kernel_ms,
        "roofline": {"bound": "mfma" if 4 * (N + 1) >= PEAK_INT8_TOPS / PEAK_HBM_GBS * 1e3 else "hbm",
                     "achieved": achieved_tops, "peak": PEAK_INT8_TOPS, "unit": "TOP/s",
                     "frac": achieved_tops / PEAK_INT8_TOPS, "traffic": traffic,
                     "algorithmic_bytes": in_bytes + out_bytes,
                     "hbm_gbs_algorithmic": (in_bytes + out_bytes) / (kernel_ms / 1e3) / 1e9},
        "cpu_baseline": cpu,
    }
    print(json.dumps(rec), flush=True)
    plan.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
