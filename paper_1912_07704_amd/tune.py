"""Autotuner of the forward's strategy (paper, "Design of the API": the
strategy decides how input data are split and processed on the GPU).

For one integer plan signature it times the shift-and-sum step of every
candidate strategy -- kernel variant x DM tile x time tile (256 or 512
output samples per workgroup) x channels per LDS stage -- on the current
device, checks that every candidate's output is
bit-identical to the first one's, and keeps the fastest.  Beams of one plan
class (same band, sampling and DM plan, any length) share one tuned
strategy (class_strategy).  Float32 plans tune the rows per LDS stage of
the forward plus adjoint (tune_f32).  Results are cached per (plan
signature, device) in a JSON file (``DD_TUNE_CACHE``, default
``~/.cache/paper_1912_07704_amd/tune.json``).  A table of strategies
measured on MI355X for the standard workloads ships with the package
(``strategies.json``) and is consulted after the user cache, so a fresh
machine does not re-time known plans.  Float32 candidates are the direct
sums at each stage size and sub-band reuse (variant 3).
"""
from __future__ import annotations

import hashlib
import json
import os
import statistics

from . import DDError, Plan, dedisperse, workspace

DD_ERR_INVALID = -2
DD_ERR_EMPTY_OUTPUT = -3

VARIANTS = (1, 2)
DM_TILES = (64, 32)
STAGES = (16, 8, 4)
TIME_TILES = (512, 256)
# variant 3 (exact sub-band reuse): its own DM tiles and time tiles (256
# samples only for the 16-wavefront tiles of 192 and 128 DMs); stages of one
# or two 8-channel sub-bands
SUBBAND = [(192, 16, 256), (192, 8, 256), (128, 16, 256), (128, 8, 256), (96, 16, 512),
           (96, 16, 256), (64, 16, 512), (64, 16, 256)]


def candidates():
    c = [{"variant": v, "dm_tile": d, "stage_chans": s, "time_tile": t}
         for v in VARIANTS for d in DM_TILES for s in STAGES for t in TIME_TILES]
    c += [{"variant": 3, "dm_tile": d, "stage_chans": s, "time_tile": t} for d, s, t in SUBBAND]
    return c


def _cache_path() -> str:
    return os.environ.get("DD_TUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "paper_1912_07704_amd",
                                       "tune.json"))


def device_arch() -> str:
    """The current device's architecture (e.g. "gfx950"): strategies are
    kept per architecture, not per marketing name."""
    import torch
    if not torch.cuda.is_available():
        return "cpu"
    return torch.cuda.get_device_properties(torch.cuda.current_device()).gcnArchName.split(":")[0]


def signature(freqs, tsamp, nsamp, ranges, dtype="u8", device=None) -> str:
    import numpy as np
    dev = device or device_arch()
    f = np.ascontiguousarray(freqs, dtype=np.float64)
    key = json.dumps({"freqs": hashlib.sha1(f.tobytes()).hexdigest(), "nchans": int(f.size),
                      "tsamp": float(tsamp), "nsamp": int(nsamp),
                      "ranges": [[float(a), float(b), float(c), int(d)] for a, b, c, d in ranges],
                      "dtype": dtype, "device": dev}, sort_keys=True)
    return hashlib.sha1(key.encode()).hexdigest()


SHIPPED = os.path.join(os.path.dirname(os.path.abspath(__file__)), "strategies.json")


def _load(path=None) -> dict:
    try:
        with open(path or _cache_path()) as fh:
            return json.load(fh)
    except (OSError, ValueError):
        return {}


def lookup(sig: str):
    """(best options, timings, source) from the user cache or the shipped
    table, or None."""
    for source, path in (("cache", None), ("shipped", SHIPPED)):
        entry = _load(path).get(sig)
        if entry:
            return entry["best"], [tuple(t) for t in entry["timings"]], source
    return None


def _store(cache: dict) -> None:
    path = _cache_path()
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        tmp = path + ".tmp"
        with open(tmp, "w") as fh:
            json.dump(cache, fh, indent=1, sort_keys=True)
        os.replace(tmp, path)
    except OSError:
        pass


def tune(freqs, tsamp, nsamp, ranges, x=None, reps: int = 3, cands=None, use_cache=True):
    """Time each candidate strategy on the device and return (best options,
    [(options, median ms of the shift-and-sum step), ...]).  `x` is a device
    uint8 [nchans, nsamp] input; a seeded uniform one is drawn if None."""
    import torch
    sig = signature(freqs, tsamp, nsamp, ranges)
    if use_cache:
        hit = lookup(sig)
        if hit:
            return hit[0], hit[1]
    if x is None:
        g = torch.Generator(device="cuda")
        g.manual_seed(0)
        x = torch.randint(0, 256, (len(freqs), nsamp), generator=g, device="cuda",
                          dtype=torch.int32).to(torch.uint8)
    timings, ref, best = [], None, None
    for opts in (cands or candidates()):
        try:
            plan = Plan(freqs, tsamp, nsamp, ranges, "u8", **opts)
        except DDError as e:
            if e.status != DD_ERR_INVALID:
                raise
            continue                 # a candidate whose tiles do not fit this plan
        ws = workspace(plan, x.device)
        out = torch.empty(plan.out_elems, dtype=torch.int32, device=x.device)
        dedisperse(x, plan, out=out, ws=ws)
        torch.cuda.synchronize()
        if ref is None:
            ref = out.clone()
        elif not torch.equal(out, ref):
            raise RuntimeError(f"strategy {opts} changed the integer result")
        ms = []
        for _ in range(reps):
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record()
            dedisperse(x, plan, out=out, ws=ws, step="sum")
            b.record()
            torch.cuda.synchronize()
            ms.append(a.elapsed_time(b))
        med = statistics.median(ms)
        timings.append((dict(opts), med))
        if best is None or med < best[1]:
            best = (dict(opts), med)
        plan.close()
        del ws, out
    if best is None:
        raise RuntimeError("no feasible strategy")
    if use_cache:
        cache = _load()
        cache[sig] = {"best": best[0], "timings": timings}
        _store(cache)
    return best[0], timings


def class_signature(freqs, tsamp, ranges, dtype="u8", device=None) -> str:
    """Signature of a plan class: the channel frequencies, sampling time, DM
    plan and device, without the series length (beams of one class differ
    only in length, which does not move the best strategy)."""
    import numpy as np
    dev = device or device_arch()
    f = np.ascontiguousarray(freqs, dtype=np.float64)
    key = json.dumps({"class": True, "freqs": hashlib.sha1(f.tobytes()).hexdigest(),
                      "nchans": int(f.size), "tsamp": float(tsamp),
                      "ranges": [[float(a), float(b), float(c), int(d)] for a, b, c, d in ranges],
                      "dtype": dtype, "device": dev}, sort_keys=True)
    return hashlib.sha1(key.encode()).hexdigest()


def class_strategy(freqs, tsamp, ranges, nsamp_probe: int = 1 << 17, reps: int = 3,
                   use_cache: bool = True):
    """(best options, source) for a plan class: from the user cache or the
    shipped table, else tuned now on a seeded input of nsamp_probe samples
    (doubled until every range has output) and cached."""
    sig = class_signature(freqs, tsamp, ranges)
    if use_cache:
        hit = lookup(sig)
        if hit:
            return hit[0], hit[2]
    nsamp = int(nsamp_probe)
    while True:
        try:
            Plan(freqs, tsamp, nsamp, ranges, "u8").close()
            break
        except DDError as e:
            if e.status != DD_ERR_EMPTY_OUTPUT or nsamp >= 1 << 24:
                raise
            nsamp *= 2
    best, timings = tune(freqs, tsamp, nsamp, ranges, reps=reps, use_cache=False)
    if use_cache:
        cache = _load()
        cache[sig] = {"best": best, "timings": timings, "probe_nsamp": nsamp}
        _store(cache)
    return best, "measured"


# float32 plans: rows staged in LDS per step (the LDS budget may lower it)
F32_STAGES = (16, 12, 8, 4, 2)


def tune_f32(freqs, tsamp, nsamp, ranges, reps: int = 5, stages=F32_STAGES, use_cache=True):
    """Time the float32 forward plus adjoint of every stage size on the
    device and return (best options, [(options, median ms), ...]).  Stage
    sizes change the order of the float32 sums, so each candidate's forward
    must agree with the first one's within 1e-5 normwise (the float32
    tolerance) instead of bit for bit.  Cached like tune()."""
    import torch
    from . import adjoint
    sig = signature(freqs, tsamp, nsamp, ranges, dtype="f32")
    if use_cache:
        hit = lookup(sig)
        if hit:
            return hit[0], hit[1]
    g = torch.Generator(device="cuda")
    g.manual_seed(0)
    x = torch.randn((len(freqs), nsamp), generator=g, device="cuda")
    timings, ref, best, seen = [], None, None, set()
    # direct sums at each stage size, then sub-band reuse (variant 3, whose
    # stage is fixed)
    for st, variant in [(st, 1) for st in stages] + [(0, 3)]:
        try:
            plan = Plan(freqs, tsamp, nsamp, ranges, "f32", variant=variant,
                        **({"stage_chans": st} if st else {}))
        except DDError as e:
            if e.status != DD_ERR_INVALID:
                raise
            continue                 # sub-band tables beyond the LDS
        key = (variant, plan.strategy["chans_stage"])
        if key in seen:                  # clamped to a stage size already timed
            plan.close()
            continue
        seen.add(key)
        ws = workspace(plan, x.device)
        out = dedisperse(x, plan, ws=ws)
        gout = torch.randn(plan.out_elems, generator=g, device="cuda")
        adjoint(gout, plan, x=x, ws=ws)
        torch.cuda.synchronize()
        if ref is None:
            ref = out.clone()
        else:
            nw = float((out - ref).abs().max() / ref.abs().max().clamp_min(1e-30))
            if nw > 1e-5:
                raise RuntimeError(f"stage {st} moved the float32 forward by {nw:.2e} normwise")
        ms = []
        for _ in range(reps):
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record()
            dedisperse(x, plan, out=out, ws=ws)
            adjoint(gout, plan, x=x, ws=ws)
            b.record()
            torch.cuda.synchronize()
            ms.append(a.elapsed_time(b))
        med = statistics.median(ms)
        opts = {"variant": key[0], "stage_chans": key[1]} if key[0] == 1 else {"variant": 3}
        timings.append((opts, med))
        if best is None or med < best[1]:
            best = (opts, med)
        plan.close()
        del ws, out, gout
    if use_cache:
        cache = _load()
        cache[sig] = {"best": best[0], "timings": timings}
        _store(cache)
    return best[0], timings


def tuned_plan(freqs, tsamp, nsamp, ranges, x=None, **kw) -> Plan:
    """A u8 plan with the fastest strategy for this device (tuned once,
    then read from the cache)."""
    best, _ = tune(freqs, tsamp, nsamp, ranges, x=x, **kw)
    return Plan(freqs, tsamp, nsamp, ranges, "u8", **best)
