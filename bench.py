#!/usr/bin/env python3
"""Benchmark of brute-force incoherent dedispersion on one MI355X.

Workload: the SKA-like single beam -- 4096 channels of uint8 over 1670 ->
1370 MHz, tsamp 64 us, 2^18 samples, a five-range DM plan up to DM 2000
(steps 0.1/0.2/0.5/1/2 with 1/2/4/8/16x time binning, 3650 trials), int32
output; synthetic N(128, 16) noise with five injected dispersed pulses.

One step is one whole forward (binning + shift-and-sum over every range)
with the input already resident in HBM.  Prints one JSON line.

    python bench.py [--steps K] [--warmup W] [--gpus 1]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("DM-trial·samples/s & ×realtime, 4096-ch uint8; fwd+bwd vs plain; "
          "HBM % peak")
UNIT = "DM-trial·samples/s"
# Integer-add roof: 256 CUs x 64 lanes x 2.4 GHz x 2 adds per lane-cycle
# (one v_add3_u32), i.e. 78.6 T adds/s.
ALU_PEAK_TOPS = 256 * 64 * 2.4e9 * 2 / 1e12
HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_dedisp_u8_ska-4096ch_traffic.json")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_1912_07704_amd", "csrc", f)
                  for f in ("dedisp.hip", "plan.h", "plan.cpp")]


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic():
    """HBM bytes per launch of the shift-and-sum kernel from the committed
    rocprofv3 FETCH_SIZE / WRITE_SIZE summary, if it was taken on the
    current kernel source; else None."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("source_hash") != kernel_source_hash():
        return None
    return t.get("bytes_per_launch")


def cpu_baseline(w, x, target_s: float):
    """Time the C oracle on a bounded sample of the workload: the first DM
    trials of the native-resolution range, all channels and samples."""
    from oracle import cref
    from oracle import dedisp as O

    rg = w.ranges[0]
    plan = O.expand_plan(w.freqs, w.tsamp, w.nsamp, [rg])
    nout = plan[0].nout
    threads = cref.max_threads()
    n = 4
    t = time.perf_counter()
    cref.dedisperse_u8_rows(x, w.freqs, w.tsamp, rg, 0, n, nout)
    dt = time.perf_counter() - t
    n = int(min(len(plan[0].dms), max(n, n * target_s / max(dt, 1e-3))))
    log(f"cpu baseline: {n} DM trials on {threads} threads")
    t = time.perf_counter()
    cref.dedisperse_u8_rows(x, w.freqs, w.tsamp, rg, 0, n, nout)
    dt = time.perf_counter() - t
    return {"value": n * nout / dt, "unit": UNIT, "cores": threads, "kind": "oracle",
            "seconds": round(dt, 3),
            "sample": (f"DM trials 0..{n - 1} of the native-resolution range (DM 0-150 step "
                       f"0.1), all {w.nchans} channels, all {nout} output samples; plain C "
                       f"oracle, OpenMP over DM trials")}


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(--gpus must be 1)", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    import paper_1912_07704_amd as dd
    import synth

    w = synth.ska_single_beam()
    log("generating input", w.name)
    x = w.make_input()
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    xt = torch.from_numpy(x).to(dev)

    t = time.perf_counter()
    plan = dd.Plan(w.freqs, w.tsamp, w.nsamp, w.ranges)
    t_plan = time.perf_counter() - t
    t = time.perf_counter()
    plan.prepare()
    torch.cuda.synchronize()
    t_upload = time.perf_counter() - t
    ws = dd.workspace(plan, dev)
    out = torch.empty(plan.out_elems, dtype=torch.int32, device=dev)
    stream = torch.cuda.current_stream()

    log("warmup", args.warmup)
    for _ in range(args.warmup):
        dd.dedisperse(xt, plan, out=out, ws=ws)
    torch.cuda.synchronize()

    # Timed region: K whole steps.
    log("timing", args.steps, "steps")
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    wall = time.perf_counter()
    e0.record(stream)
    for _ in range(args.steps):
        dd.dedisperse(xt, plan, out=out, ws=ws)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall
    ms_step = e0.elapsed_time(e1) / args.steps

    # The dominant kernel alone (dd_forward_sum is one launch of the
    # shift-and-sum kernel), and the binning step alone, each bracketed by
    # events on the launch stream.
    def per_launch(fn, n):
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(n)]
        for a, b in ev:
            a.record(stream)
            fn()
            b.record(stream)
        torch.cuda.synchronize()
        return [a.elapsed_time(b) for a, b in ev]

    n_k = max(5, args.steps)
    t_sum = per_launch(lambda: dd.dedisperse(xt, plan, out=out, ws=ws, step="sum"), n_k)
    t_bin = per_launch(lambda: dd.bin_input(xt, plan, ws), n_k)
    ms_sum = float(np.mean(t_sum))
    ms_bin = float(np.mean(t_bin))

    samples = plan.out_elems                              # sum_r ndms_r * nout_r
    value = samples / (ms_step / 1e3)
    adds = sum(r.ndms * r.nout for r in plan.ranges) * w.nchans
    achieved = adds / (ms_sum / 1e3) / 1e12
    traffic = measured_traffic()
    alg_bytes = w.nchans * w.nsamp + samples * 4          # one input read + the output
    realtime = (w.nsamp - plan.overlap) * w.tsamp / (ms_step / 1e3)

    res = {
        "metric": METRIC,
        "value": value,
        "unit": UNIT,
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u8",
        "data": "synthetic",
        "config": {"workload": w.name, "nchans": w.nchans, "nsamp": w.nsamp,
                   "tsamp_us": w.tsamp * 1e6, "band_mhz": [1670.0, 1370.0],
                   "dm_ranges": [list(r) for r in w.ranges], "ndms": plan.ndms_total,
                   "output": "int32", "dm_trial_samples": samples},
        "x_realtime": realtime,
        "x_realtime_full_chunk": w.nsamp * w.tsamp / (ms_step / 1e3),
        "roofline": {"bound": "alu", "achieved": achieved, "peak": ALU_PEAK_TOPS,
                     "unit": "TOP/s", "frac": achieved / ALU_PEAK_TOPS, "traffic": traffic,
                     "kernel": "k_dedisp_u8", "kernel_ms": ms_sum,
                     "adds_per_launch": adds, "algorithmic_bytes_per_launch": alg_bytes,
                     "algorithmic_hbm_gbs": alg_bytes / (ms_sum / 1e3) / 1e9,
                     "hbm_frac_of_peak": (traffic / (ms_sum / 1e3) / 1e9 / HBM_PEAK_GBS
                                          if traffic else None)},
        "steps_ms": {"bin": ms_bin, "sum": ms_sum, "plan_create_s": t_plan,
                     "table_upload_s": t_upload, "wall_s": wall},
    }
    if not args.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline(w, x, args.cpu_seconds)
    print(json.dumps(res), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
