"""Parity of the HIP integer forward with the CPU oracle (bit-exact int32).

Every call goes through the C ABI (dd_forward / dd_forward_bin /
dd_forward_sum) on cuda:0.  Each test prints its case before touching the
GPU so a failing run names it.
"""
import os

import numpy as np
import pytest

import synth
from oracle import cref
from oracle import dedisp as O

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
dd = pytest.importorskip("paper_1912_07704_amd")


def say(*a):
    print("[case]", *a, flush=True)


# the library default (variant 3 where its patterns fit the LDS, else the
# direct kernel) and both direct variants at both time tiles
STRATEGIES = {"default": {}, "v1": {"variant": 1}, "v2": {"variant": 2},
              "v1-t256": {"variant": 1, "time_tile": 256}, "v2-t256": {"variant": 2, "time_tile": 256}}


def gpu_forward(x, freqs, tsamp, ranges, out_extra=0, canary=-123456789, opts=None):
    plan = dd.Plan(freqs, tsamp, x.shape[1], ranges, **(opts or {}))
    xt = torch.from_numpy(np.ascontiguousarray(x)).cuda()
    out = torch.full((plan.out_elems + out_extra,), canary, dtype=torch.int32, device="cuda")
    dd.dedisperse(xt, plan, out=out)
    torch.cuda.synchronize()
    return out.cpu().numpy(), plan


_ORACLE = {}


def oracle_flat(x, freqs, tsamp, ranges):
    key = (x.shape, x.tobytes().__hash__(), tuple(np.asarray(freqs).tolist()), tsamp,
           tuple(map(tuple, ranges)))
    if key not in _ORACLE:
        if x.shape[0] * x.shape[1] <= 2_000_000 and len(ranges) <= 3:
            outs, _ = O.dedisperse(x, freqs, tsamp, ranges)
            _ORACLE[key] = O.concat(outs)
        else:
            _ORACLE[key] = cref.dedisperse_u8(x, freqs, tsamp, ranges).astype(np.int64)
    return _ORACLE[key]


def test_tiny_workload_bit_exact():
    w = synth.tiny()
    say("tiny", w.name)
    x = w.make_input()
    got, plan = gpu_forward(x, w.freqs, w.tsamp, w.ranges, out_extra=1000)
    want = cref.dedisperse_u8(x, w.freqs, w.tsamp, w.ranges)
    assert np.array_equal(got[: plan.out_elems], want)
    assert (got[plan.out_elems:] == -123456789).all(), "wrote past out_elems"


def random_case(seed):
    rng = np.random.default_rng(1000 + seed)
    while True:
        nch = int(rng.integers(1, 300))
        nsamp = int(rng.integers(64, 8193))
        f_top = float(rng.uniform(1000.0, 1700.0))
        bw = float(rng.uniform(10.0, 400.0))
        freqs = synth.band_freqs(f_top, f_top - bw, nch)
        if seed % 3 == 1:
            freqs = freqs[::-1].copy()          # ascending band
        if seed % 5 == 2:
            freqs = rng.permutation(freqs)      # arbitrary channel order
        tsamp = float(rng.choice([64e-6, 2.56e-4, 1e-3]))
        ranges, lo = [], 0.0
        for _ in range(int(rng.integers(1, 4))):
            step = float(rng.choice([0.1, 0.5, 1.0, 3.0]))
            n = int(rng.integers(1, 80))
            ranges.append((lo, lo + n * step, step, int(rng.choice([1, 2, 3, 4, 6, 8, 16]))))
            lo += n * step
        try:
            O.expand_plan(freqs, tsamp, nsamp, ranges)
        except ValueError:
            continue
        x = rng.integers(0, 256, size=(nch, nsamp)).astype(np.uint8)
        return x, freqs, tsamp, ranges


@pytest.mark.parametrize("strategy", sorted(STRATEGIES))
@pytest.mark.parametrize("seed", range(16))
def test_random_shapes_bit_exact(seed, strategy):
    x, freqs, tsamp, ranges = random_case(seed)
    say("random", seed, strategy, x.shape, ranges)
    got, plan = gpu_forward(x, freqs, tsamp, ranges, out_extra=64, opts=STRATEGIES[strategy])
    assert np.array_equal(got[: plan.out_elems], oracle_flat(x, freqs, tsamp, ranges))
    assert (got[plan.out_elems:] == -123456789).all()


# variant 3 at every workgroup shape it accepts: (DM tile, time tile)
SUBBAND_SHAPES = [(192, 256), (128, 256), (96, 512), (96, 256), (64, 512), (64, 256)]


@pytest.mark.parametrize("dm_tile,time_tile", SUBBAND_SHAPES)
def test_subband_shapes_bit_exact(dm_tile, time_tile):
    """Random shapes through variant 3 at each of its workgroup shapes (the
    shapes whose sub-band patterns exceed the LDS are skipped; at least a
    few must fit)."""
    ran = 0
    for seed in range(12):
        x, freqs, tsamp, ranges = random_case(100 + seed)
        try:
            plan = dd.Plan(freqs, tsamp, x.shape[1], ranges, "u8", variant=3, dm_tile=dm_tile,
                           time_tile=time_tile)
        except dd.DDError:
            continue                                # patterns beyond the LDS
        plan.close()
        say("subband", dm_tile, time_tile, seed, x.shape, ranges)
        got, plan = gpu_forward(x, freqs, tsamp, ranges, out_extra=64,
                                opts={"variant": 3, "dm_tile": dm_tile, "time_tile": time_tile})
        assert plan.strategy["time_tile"] == time_tile and plan.strategy["dm_tile"] == dm_tile
        assert np.array_equal(got[: plan.out_elems], oracle_flat(x, freqs, tsamp, ranges))
        assert (got[plan.out_elems:] == -123456789).all()
        ran += 1
    assert ran >= 3


EDGES = {
    # one channel: the output is the binned input itself
    "one_channel": (1, 300, [(0.0, 5.0, 1.0, 1), (5.0, 7.0, 1.0, 3)]),
    # odd channel count with a partial LDS stage, a partial DM tile (33 DMs)
    "odd_channels_partial_dm_tile": (17, 2000, [(0.0, 33.0, 1.0, 1)]),
    # exactly one DM, exactly one valid output sample
    "single_dm_single_sample": (8, 0, [(40.0, 41.0, 1.0, 1)]),
    # the largest binning factor of the integer path
    "downsample_256": (6, 6000, [(0.0, 2.0, 1.0, 256)]),
    # binning cascades: 6 from 2 (factor 3), 9 from 3 and 12 from 6
    "cascade": (40, 3000, [(0.0, 10.0, 1.0, 2), (10.0, 20.0, 1.0, 6), (20.0, 30.0, 2.0, 3),
                           (30.0, 40.0, 2.0, 9), (40.0, 50.0, 2.0, 12)]),
    # a DM tile whose delay spread is large (coarse step, low frequencies)
    "wide_spread": (64, 20000, [(0.0, 400.0, 12.5, 1)]),
}


@pytest.mark.parametrize("strategy", sorted(STRATEGIES))
@pytest.mark.parametrize("name", sorted(EDGES))
def test_edge_cases_bit_exact(name, strategy):
    nch, nsamp, ranges = EDGES[name]
    freqs = synth.band_freqs(1500.0, 1200.0, nch) if nch > 1 else np.array([1400.0])
    tsamp = 1e-3
    if name == "single_dm_single_sample":
        s = O.shift_table(freqs, tsamp, [40.0])
        nsamp = int(s.max()) + 1
    if name == "wide_spread":
        freqs = synth.band_freqs(500.0, 300.0, nch)
        tsamp = 1e-3
    rng = np.random.default_rng(hash(name) % 2**32)
    x = rng.integers(0, 256, size=(nch, nsamp)).astype(np.uint8)
    if name == "downsample_256":
        x[:] = 255                               # the largest binned value, 255*256
    say("edge", name, strategy, x.shape, ranges)
    got, plan = gpu_forward(x, freqs, tsamp, ranges, out_extra=8, opts=STRATEGIES[strategy])
    want = oracle_flat(x, freqs, tsamp, ranges)
    assert np.array_equal(got[: plan.out_elems], want)
    if name == "single_dm_single_sample":
        assert plan.out_elems == 1


@pytest.mark.parametrize("strategy", sorted(STRATEGIES))
def test_all_255_and_all_zero_extremes(strategy):
    """Saturated input: every sum reaches its bound (255*nchans*ds) without a
    carry between the packed 16-bit halves."""
    freqs = synth.band_freqs(1670.0, 1370.0, 1024)
    ranges = [(0.0, 40.0, 1.0, 1), (40.0, 80.0, 2.0, 16)]
    for val in (255, 0):
        x = np.full((1024, 8192), val, dtype=np.uint8)
        say("extreme", val, strategy)
        got, plan = gpu_forward(x, freqs, 64e-6, ranges, opts=STRATEGIES[strategy])
        outs = plan.split(got)
        assert (outs[0] == 255 * 1024 * (val // 255)).all()
        assert (outs[1] == 255 * 1024 * 16 * (val // 255)).all()


def test_steps_compose_and_repeat_bit_identically():
    w = synth.ska_single_beam(nsamp=1 << 15, nchans=512)
    say("steps", w.name)
    x = torch.from_numpy(w.make_input()).cuda()
    plan = dd.Plan(w.freqs, w.tsamp, w.nsamp, w.ranges)
    ws = dd.workspace(plan)
    a = dd.dedisperse(x, plan, ws=ws)
    dd.bin_input(x, plan, ws)
    b = dd.dedisperse(x, plan, ws=ws, step="sum")
    c = dd.dedisperse(x, plan)
    torch.cuda.synchronize()
    assert torch.equal(a, b) and torch.equal(a, c)
    want = cref.dedisperse_u8(w.make_input(), w.freqs, w.tsamp, w.ranges)
    assert np.array_equal(a.cpu().numpy(), want)


def test_other_stream():
    w = synth.tiny()
    say("stream", w.name)
    x = torch.from_numpy(w.make_input()).cuda()
    plan = dd.Plan(w.freqs, w.tsamp, w.nsamp, w.ranges)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        out = dd.dedisperse(x, plan)
    s.synchronize()
    want = cref.dedisperse_u8(w.make_input(), w.freqs, w.tsamp, w.ranges)
    assert np.array_equal(out.cpu().numpy(), want)


def test_forced_allocation_failure_is_reported():
    w = synth.tiny()
    say("fault-hook alloc")
    plan = dd.Plan(w.freqs, w.tsamp, w.nsamp, w.ranges)
    x = torch.zeros((w.nchans, w.nsamp), dtype=torch.uint8, device="cuda")
    os.environ["DD_FAULT"] = "alloc"
    try:
        with pytest.raises(dd.DDError) as e:
            dd.dedisperse(x, plan)
        assert e.value.status == -8
    finally:
        del os.environ["DD_FAULT"]
    out = dd.dedisperse(x, plan)           # the plan is still usable
    torch.cuda.synchronize()
    assert int(out.abs().max()) == 0


# ---------------------------------------------------------------------------
# Full-size SKA-like beam (the benchmark's workload and launch configuration)
# ---------------------------------------------------------------------------

@pytest.fixture(scope="module")
def ska():
    w = synth.ska_single_beam()
    say("ska full size: generating input")
    x = w.make_input()
    plan = dd.Plan(w.freqs, w.tsamp, w.nsamp, w.ranges)
    xt = torch.from_numpy(x).cuda()
    say("ska full size: forward")
    out = dd.dedisperse(xt, plan)
    torch.cuda.synchronize()
    return w, x, plan, out


@pytest.fixture(scope="module")
def ska_want(ska):
    w, x, plan, out = ska
    say("ska whole output: C oracle on", cref.max_threads(), "threads")
    return cref.dedisperse_u8(x, w.freqs, w.tsamp, w.ranges)


def test_ska_full_size_whole_output_bit_exact(ska, ska_want):
    """Every one of the 536 529 400 outputs of the default strategy (the
    launch configuration the benchmark times) against the plain C oracle
    over the whole plan."""
    w, x, plan, out = ska
    want = ska_want
    say("ska whole output: compare")
    got = out.cpu().numpy()
    assert got.shape == want.shape
    bad = np.flatnonzero(got != want)
    assert bad.size == 0, f"{bad.size} outputs differ, first at {bad[:8]}"


def tile_edge_rows(ndms, dm_tile, wave_dms=(8, 12)):
    """Rows at every DM-tile edge (first, second, last two of each tile),
    the first rows of a few wavefronts, and the range's last rows."""
    rows = {ndms - 2, ndms - 1, ndms // 2}
    for t0 in range(0, ndms, dm_tile):
        rows |= {t0, t0 + 1, t0 + dm_tile - 2, t0 + dm_tile - 1}
        for wd in wave_dms:
            rows |= {t0 + wd - 1, t0 + wd}
    return sorted(r for r in rows if 0 <= r < ndms)


def test_ska_full_size_rows_bit_exact(ska, ska_want):
    """Whole rows at the edges of the default strategy's DM tiles (and of
    the direct kernel's 32/64-DM tiles) in every range, including the partial
    last tile, against the C oracle: rows of the whole-plan reference, and
    for range 0 the oracle's row-by-row entry as well."""
    w, x, plan, out = ska
    outs = plan.split(out)
    wants = plan.split(ska_want)
    dm_tile = plan.strategy["dm_tile"]
    for r, (rg, ri) in enumerate(zip(w.ranges, plan.ranges)):
        rows = sorted(set(tile_edge_rows(ri.ndms, dm_tile)) | {31, 32, 33, 63, 64})
        say("ska rows", r, rows)
        got = outs[r][torch.tensor(rows, device="cuda")].cpu().numpy()
        for i, d in enumerate(rows):
            assert np.array_equal(got[i], wants[r][d]), (r, d)
        if r == 0:
            for d in (dm_tile - 1, dm_tile, ri.ndms - 1):
                want = cref.dedisperse_u8_rows(x, w.freqs, w.tsamp, rg, d, d + 1, ri.nout)[0]
                assert np.array_equal(got[rows.index(d)], want), (r, d)


def test_ska_full_size_sampled_outputs(ska):
    w, x, plan, out = ska
    op = O.expand_plan(w.freqs, w.tsamp, w.nsamp, w.ranges)
    outs = plan.split(out)
    rng = np.random.default_rng(77)
    for r, ri in enumerate(plan.ranges):
        d = rng.integers(0, ri.ndms, 300)
        t = rng.integers(0, ri.nout, 300)
        t[:20] = ri.nout - 1 - np.arange(20)          # the ragged end of the last tile
        say("ska samples", r)
        got = outs[r][torch.from_numpy(d).cuda(), torch.from_numpy(t).cuda()].cpu().numpy()
        assert np.array_equal(got, O.dedisperse_at(x, op, r, d, t))


def test_ska_pulses_recovered(ska):
    w, x, plan, out = ska
    outs = plan.split(out)
    dms = plan.dms()
    f = w.freqs
    dmax = 1.0 / f.min() ** 2 - 1.0 / f.max() ** 2
    for p in w.pulses:
        r = next(i for i, rg in enumerate(w.ranges) if rg[0] <= p.dm < rg[1])
        ri = plan.ranges[r]
        ds = ri.downsample
        o = outs[r].double()
        o = o - o.mean(dim=1, keepdim=True)
        wb = max(1, -(-p.width // ds))
        cs = torch.nn.functional.pad(torch.cumsum(o, dim=1), (1, 0))
        box = cs[:, wb:] - cs[:, :-wb]
        lo = max(0, p.t0 // ds - 300)
        hi = min(box.shape[1], p.t0 // ds + 300)
        sub = box[:, lo:hi]
        k = int(torch.argmax(sub))
        d, t = divmod(k, sub.shape[1])
        dm_found = dms[sum(q.ndms for q in plan.ranges[:r]) + d]
        tol = 1.5 * (w.ranges[r][2] + p.width * w.tsamp / (O.K_DM * dmax))
        say("pulse", p, dm_found, (t + lo) * ds)
        assert abs(dm_found - p.dm) <= tol
        assert abs((t + lo) * ds - p.t0) <= p.width + ds


@pytest.mark.parametrize("seed", range(6))
def test_fused_binning_levels_bit_exact(seed):
    """nsamp a multiple of 16, so downsamples 1, 2, 4, 8 and 16 are binned in
    one pass over the input, next to 3, 6 and 32 (binned from their source
    levels): bit-exact against the oracle for both integer kernels."""
    rng = np.random.default_rng(3000 + seed)
    nch = int(rng.integers(1, 200))
    nsamp = 16 * int(rng.integers(300, 1500))
    dss = sorted(int(d) for d in rng.choice([1, 2, 4, 8, 16, 3, 6, 32],
                                            size=int(rng.integers(1, 6)), replace=False))
    ranges, lo = [], 0.0
    for ds in dss:
        n = int(rng.integers(5, 40))
        ranges.append((lo, lo + n * 0.5, 0.5, ds))
        lo += n * 0.5
    freqs = synth.band_freqs(1500.0, 1300.0, nch)
    tsamp = 2.56e-4
    x = rng.integers(0, 256, size=(nch, nsamp)).astype(np.uint8)
    say("fused binning", seed, x.shape, ranges)
    want = oracle_flat(x, freqs, tsamp, ranges)
    for variant in (1, 3):
        try:
            plan = dd.Plan(freqs, tsamp, nsamp, ranges, "u8", variant=variant)
        except dd.DDError:
            continue                                # variant 3 beyond the LDS
        xt = torch.from_numpy(x).cuda()
        out = dd.dedisperse(xt, plan)
        torch.cuda.synchronize()
        assert np.array_equal(out.cpu().numpy(), want), variant
