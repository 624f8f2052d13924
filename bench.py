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
import re
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
# rocprofv3 FETCH_SIZE/WRITE_SIZE summary of the shift-and-sum kernel, per kernel
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "{kernel}_ska-4096ch_traffic.json")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_1912_07704_amd", "csrc", f)
                  for f in ("dedisp.hip", "plan.h", "plan.cpp")]


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def _code_only(text: str) -> str:
    """C++ source without its comments and blank lines (a comment edit does
    not change what the counters measured)."""
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    lines = []
    for line in text.splitlines():
        code = line.split("//", 1)[0].rstrip()
        if code.strip():
            lines.append(code)
    return "\n".join(lines)


def kernel_source_hash() -> str:
    """First 16 hex digits of the sha256 of the kernel sources' code (the
    shift-and-sum kernels, the plan tables they read)."""
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(f, encoding="utf-8") as fh:
            h.update(_code_only(fh.read()).encode())
    return h.hexdigest()[:16]


def kernel_name(strategy) -> str:
    """The shift-and-sum kernel a strategy launches."""
    return "k_dedisp_u8_sb" if strategy["variant"] == 3 else "k_dedisp_u8"


def measured_traffic(kernel):
    """HBM bytes per launch of the shift-and-sum kernel from the committed
    rocprofv3 FETCH_SIZE / WRITE_SIZE summary, if it was taken on the
    current kernel source; else None."""
    try:
        with open(TRAFFIC_FILE.format(kernel=kernel)) as f:
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
    cref.dedisperse_u8_rows(x, w.freqs, w.tsamp, rg, 0, 1, nout)      # thread pool warm-up
    n = 2 * threads               # the probe keeps every thread busy (OpenMP over DM trials)
    t = time.perf_counter()
    cref.dedisperse_u8_rows(x, w.freqs, w.tsamp, rg, 0, n, nout)
    dt = time.perf_counter() - t
    n = int(min(len(plan[0].dms), max(n, n * target_s / max(dt, 1e-3))))
    log(f"cpu baseline: {n} DM trials on {threads} threads")
    t = time.perf_counter()
    cref.dedisperse_u8_rows(x, w.freqs, w.tsamp, rg, 0, n, nout)
    dt = time.perf_counter() - t
    # the same oracle on one thread, over a few DM trials (about 3 s)
    t = time.perf_counter()
    cref.dedisperse_u8_rows(x, w.freqs, w.tsamp, rg, 0, 1, nout, threads=1)
    n1 = int(min(len(plan[0].dms), max(1, 3.0 / max(time.perf_counter() - t, 1e-3))))
    t = time.perf_counter()
    cref.dedisperse_u8_rows(x, w.freqs, w.tsamp, rg, 0, n1, nout, threads=1)
    dt1 = time.perf_counter() - t
    return {"value": n * nout / dt, "unit": UNIT, "cores": threads, "kind": "oracle",
            "seconds": round(dt, 3),
            "sample": (f"DM trials 0..{n - 1} of the native-resolution range (DM 0-150 step "
                       f"0.1), all {w.nchans} channels, all {nout} output samples; plain C "
                       f"oracle, OpenMP over DM trials"),
            "single_thread_value": n1 * nout / dt1,
            "single_thread_sample": f"DM trials 0..{n1 - 1} of the same range on 1 thread "
                                    f"({dt1:.2f} s)"}


def _time(torch, fn, n):
    ts = []
    for _ in range(n):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        fn()
        b.record()
        torch.cuda.synchronize()
        ts.append(a.elapsed_time(b))
    return sorted(ts)[len(ts) // 2]


def leg_fwdbwd(dd, synth, torch, plain_value):
    """Differentiable workload (1024 ch float32, 2^16 samples, DM 0..511):
    forward with weights, then the hand-written adjoint (dX and dw)."""
    w = synth.differentiable()
    log("leg fwd+bwd:", w.name)
    x = torch.from_numpy(w.make_input()).cuda()
    wt = torch.ones(w.nchans, device="cuda")
    plan = dd.Plan(w.freqs, w.tsamp, w.nsamp, w.ranges, "f32")
    ws = dd.workspace(plan)
    out = dd.dedisperse(x, plan, weights=wt, ws=ws)
    g = torch.randn(plan.out_elems, device="cuda",
                    generator=torch.Generator("cuda").manual_seed(w.seed))
    dd.adjoint(g, plan, x=x, weights=wt, ws=ws)
    torch.cuda.synchronize()
    f_ms = _time(torch, lambda: dd.dedisperse(x, plan, out=out, weights=wt, ws=ws), 5)
    b_ms = _time(torch, lambda: dd.adjoint(g, plan, x=x, weights=wt, ws=ws), 5)
    samples = plan.out_elems
    v = samples / ((f_ms + b_ms) / 1e3)
    return {"workload": w.name, "fwd_ms": f_ms, "bwd_ms": b_ms,
            "fwd_dm_trial_samples_per_s": samples / (f_ms / 1e3),
            "fwd_bwd_dm_trial_samples_per_s": v, "vs_plain_single_beam": v / plain_value,
            "note": "float32; plain = the uint8 single-beam value of this line"}


def leg_batched(dd, synth, torch, plain_value, opts):
    """64 uint8 beams of uneven shape in one persistent launch per kernel (inputs drawn
    on the GPU, excluded from timing)."""
    wls = synth.batched_beams()
    log("leg batched:", len(wls), "beams")
    # the single beam's tuned strategy for every beam
    o = {k: v for k, v in opts.items() if k in ("variant", "dm_tile", "stage_chans")}
    plans = [dd.Plan(w.freqs, w.tsamp, w.nsamp, w.ranges, **o) for w in wls]
    batch = dd.Batch(plans)
    batch.prepare()
    xin = torch.empty(batch.in_bytes, dtype=torch.uint8, device="cuda")
    for w, p, off in zip(wls, plans, batch.in_offsets):
        xin[off: off + p.nchans * p.nsamp] = synth.filterbank_u8_device(
            w.seed, w.freqs, w.tsamp, w.nsamp, w.pulses).reshape(-1)
    out = torch.empty(batch.out_elems, dtype=torch.int32, device="cuda")
    ws = torch.empty(batch.workspace_bytes, dtype=torch.uint8, device="cuda")
    dd.dedisperse_batch(xin, batch, out=out, ws=ws)
    torch.cuda.synchronize()
    ms = _time(torch, lambda: dd.dedisperse_batch(xin, batch, out=out, ws=ws), 3)
    samples = sum(p.out_elems for p in plans)
    v = samples / (ms / 1e3)
    res = {"workload": f"{len(wls)} uint8 beams, 1024-4096 ch, 2^16-2^18 samples, DM max "
                       "500/1000/2000", "ms": ms, "dm_trial_samples": samples,
           "dm_trial_samples_per_s": v, "vs_plain_single_beam": v / plain_value,
           "strategy": plans[0].strategy,
           "work_items": batch.work_items, "launches": "bins per beam + %d persistent" % len(
               {(p.strategy["variant"], p.strategy["dm_tile"]) for p in plans})}
    del xin, out, ws
    batch.close()
    return res


def leg_boxcar(dd, synth, torch):
    """32 float32 beams x 4096 ch x 2^17, DM 0..999: boxcar loss (out never
    stored) and its backward (out recomputed, adjoint)."""
    wls = synth.batched_differentiable()
    w0 = wls[0]
    log("leg boxcar:", len(wls), "beams")
    plan = dd.Plan(w0.freqs, w0.tsamp, w0.nsamp, w0.ranges, "f32")
    x = torch.empty((len(wls), w0.nchans, w0.nsamp), dtype=torch.float32, device="cuda")
    gen = torch.Generator(device="cuda")
    for b, w in enumerate(wls):
        gen.manual_seed(w.seed)
        x[b].normal_(generator=gen)
    wt = torch.ones(w0.nchans, device="cuda")
    ws = dd.workspace(plan)
    dd.boxcar_loss(x, plan, wt, ws=ws)
    torch.cuda.synchronize()
    l_ms = _time(torch, lambda: dd.boxcar_loss(x, plan, wt, ws=ws), 1)
    dx, dw = dd.boxcar_backward(x, plan, wt, ws=ws)
    torch.cuda.synchronize()
    b_ms = _time(torch, lambda: dd.boxcar_backward(x, plan, wt, ws=ws), 1)
    samples = plan.out_elems * len(wls)
    return {"workload": f"{len(wls)} float32 beams x 4096 ch x 2^17, DM 0..999, boxcar 1..32",
            "loss_ms": l_ms, "backward_ms": b_ms,
            "fwd_dm_trial_samples_per_s": samples / (l_ms / 1e3),
            "fwd_bwd_dm_trial_samples_per_s": samples / ((l_ms + b_ms) / 1e3)}


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-tune", action="store_true", help="use the default strategy")
    ap.add_argument("--retune", action="store_true",
                    help="time every candidate strategy instead of using the cached or "
                         "shipped strategy table")
    ap.add_argument("--copy-gib", type=float, default=0.0,
                    help="also run one device-to-device copy of this many GiB (a counter "
                         "calibration reference for profiles)")
    ap.add_argument("--legs", default="fwdbwd,batched,boxcar",
                    help="extra legs after the main one: fwdbwd,batched,boxcar (or none)")
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

    tune_info = None
    opts = {}
    if not args.no_tune:
        from paper_1912_07704_amd import tune as tuner
        t = time.perf_counter()
        sig = tuner.signature(w.freqs, w.tsamp, w.nsamp, w.ranges)
        hit = None if args.retune else tuner.lookup(sig)
        if hit:
            opts, timings, source = hit
        else:
            opts, timings = tuner.tune(w.freqs, w.tsamp, w.nsamp, w.ranges, x=xt,
                                       use_cache=False)
            source = "measured"
        tune_info = {"best": opts, "source": source, "signature": sig,
                     "device": torch.cuda.get_device_name(dev), "arch": tuner.device_arch(),
                     "seconds": round(time.perf_counter() - t, 2),
                     "candidates_sum_ms": [[o, round(m, 3)] for o, m in timings]}
        log("strategy", opts, "from", source)
    t = time.perf_counter()
    plan = dd.Plan(w.freqs, w.tsamp, w.nsamp, w.ranges, **opts)
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
    kernel = kernel_name(plan.strategy)
    traffic = measured_traffic(kernel)
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
                     "kernel": kernel, "kernel_ms": ms_sum,
                     "adds_per_launch": adds, "algorithmic_bytes_per_launch": alg_bytes,
                     "algorithmic_hbm_gbs": alg_bytes / (ms_sum / 1e3) / 1e9,
                     "hbm_frac_of_peak": (traffic / (ms_sum / 1e3) / 1e9 / HBM_PEAK_GBS
                                          if traffic else None)},
        "steps_ms": {"bin": ms_bin, "sum": ms_sum, "plan_create_s": t_plan,
                     "table_upload_s": t_upload, "wall_s": wall},
        "strategy": plan.strategy,
        "tuning": tune_info,
    }
    del out, ws
    torch.cuda.empty_cache()
    legs = [] if args.legs in ("", "none") else args.legs.split(",")
    if "fwdbwd" in legs:
        res["fwd_bwd"] = leg_fwdbwd(dd, synth, torch, value)
    if "batched" in legs:
        del xt
        torch.cuda.empty_cache()
        res["batched"] = leg_batched(dd, synth, torch, value, opts)
    if "boxcar" in legs:
        torch.cuda.empty_cache()
        res["boxcar"] = leg_boxcar(dd, synth, torch)
    if args.copy_gib > 0:
        n = int(args.copy_gib * (1 << 30))
        src = torch.empty(n, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        res["copy_reference_bytes"] = n
        del src, dst
    if not args.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline(w, x, args.cpu_seconds)
    print(json.dumps(res), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
