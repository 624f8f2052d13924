"""The autotuner (the paper's strategy, "Plan and strategy", picked by
timing candidates on the device): every feasible candidate is timed, the
winner's output equals the oracle bit for bit, and the per-device cache
round-trips."""
import json

import numpy as np
import pytest

import synth
from oracle import cref

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
dd = pytest.importorskip("paper_1912_07704_amd")
from paper_1912_07704_amd import tune  # noqa: E402


def say(*a):
    print("[case]", *a, flush=True)


def small_problem():
    freqs = synth.band_freqs(1670.0, 1370.0, 256)
    tsamp = 128e-6
    nsamp = 24576
    ranges = [(0.0, 150.0, 0.5, 1), (150.0, 300.0, 1.0, 2)]
    x = np.random.default_rng(41).integers(0, 256, size=(256, nsamp)).astype(np.uint8)
    return freqs, tsamp, nsamp, ranges, x


def test_tune_times_every_feasible_candidate_and_caches(tmp_path, monkeypatch):
    cache = tmp_path / "tune.json"
    monkeypatch.setenv("DD_TUNE_CACHE", str(cache))
    freqs, tsamp, nsamp, ranges, x = small_problem()
    xt = torch.from_numpy(x).cuda()
    say("tune: timing candidates")
    best, timings = tune.tune(freqs, tsamp, nsamp, ranges, x=xt, reps=2)
    feasible = []
    for opts in tune.candidates():
        try:
            dd.Plan(freqs, tsamp, nsamp, ranges, "u8", **opts).close()
            feasible.append(opts)
        except dd.DDError as e:
            assert e.status == tune.DD_ERR_INVALID
    assert [t[0] for t in timings] == feasible
    assert all(ms > 0 for _, ms in timings)
    assert best == min(timings, key=lambda t: t[1])[0]
    # the winner's output equals the oracle
    plan = dd.Plan(freqs, tsamp, nsamp, ranges, "u8", **best)
    out = dd.dedisperse(xt, plan)
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy(), cref.dedisperse_u8(x, freqs, tsamp, ranges))
    # the cache holds the result under the plan's signature and is read back
    sig = tune.signature(freqs, tsamp, nsamp, ranges)
    stored = json.loads(cache.read_text())[sig]
    assert stored["best"] == best
    hit = tune.lookup(sig)
    assert hit is not None and hit[0] == best and hit[2] == "cache"
    best2, timings2 = tune.tune(freqs, tsamp, nsamp, ranges, x=xt)
    assert best2 == best and [tuple(t) for t in timings2] == [tuple(t) for t in timings]
    p2 = tune.tuned_plan(freqs, tsamp, nsamp, ranges, x=xt)
    assert p2.strategy["variant"] == plan.strategy["variant"]
    assert p2.strategy["dm_tile"] == plan.strategy["dm_tile"]


def test_tune_explicit_candidates_without_cache(tmp_path, monkeypatch):
    """An explicit candidate list is timed as given, and use_cache=False
    neither reads nor writes the cache."""
    monkeypatch.setenv("DD_TUNE_CACHE", str(tmp_path / "tune.json"))
    freqs, tsamp, nsamp, ranges, x = small_problem()
    xt = torch.from_numpy(x).cuda()
    cands = [{"variant": 1, "dm_tile": 64, "stage_chans": 16},
             {"variant": 1, "dm_tile": 32, "stage_chans": 8}]
    best, timings = tune.tune(freqs, tsamp, nsamp, ranges, x=xt, reps=1, cands=cands,
                              use_cache=False)
    assert len(timings) == 2 and best in cands
    assert not (tmp_path / "tune.json").exists()     # use_cache=False writes nothing


def test_tune_f32_times_direct_and_subband_candidates(tmp_path, monkeypatch):
    """The float32 tuner times the direct sums at each stage size and
    sub-band reuse (variant 3), keeps the fastest, caches it, and the
    winner's forward is within the float32 tolerance of the oracle."""
    monkeypatch.setenv("DD_TUNE_CACHE", str(tmp_path / "tune.json"))
    freqs = synth.band_freqs(1500.0, 1200.0, 96)
    tsamp, nsamp, ranges = 2.56e-4, 6000, [(0.0, 60.0, 1.0, 1)]
    say("tune_f32")
    best, timings = tune.tune_f32(freqs, tsamp, nsamp, ranges, reps=2)
    kinds = [t[0] for t in timings]
    assert {"variant": 3} in kinds and any(k.get("variant") == 1 for k in kinds)
    assert all(ms > 0 for _, ms in timings)
    assert best == min(timings, key=lambda t: t[1])[0]
    best2, _ = tune.tune_f32(freqs, tsamp, nsamp, ranges)          # from the cache
    assert best2 == best
    x = np.random.default_rng(5).standard_normal((96, nsamp)).astype(np.float32)
    plan = dd.Plan(freqs, tsamp, nsamp, ranges, "f32", **best)
    out = dd.dedisperse(torch.from_numpy(x).cuda(), plan).cpu().numpy().astype(np.float64)
    want = cref.dedisperse_f32(x, freqs, tsamp, ranges)
    terms = cref.dedisperse_f32(np.abs(x), freqs, tsamp, ranges)
    assert np.abs(out - want).max() <= 1e-5 * np.abs(want).max()
    assert (np.abs(out - want) <= 1e-5 * terms + 1e-30).all()
