"""Host-side tests of the C ABI (no GPU): the library loads and exports every
symbol include/dd.h declares, plans match the oracle's DM grid, shift table
and sizes exactly, and every validation error is reported before any device
work."""
import ctypes
import os
import re

import numpy as np
import pytest

import synth
from oracle import dedisp as O

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dd.h")

dd = pytest.importorskip("paper_1912_07704_amd")
from paper_1912_07704_amd import _lib  # noqa: E402


def header_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(dd_[a-z_]+)\s*\(", text)))


def test_library_exports_every_header_symbol():
    L = _lib.lib()
    names = header_functions()
    assert len(names) >= 12
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(_lib.SIGNATURES), "binding and header disagree"


def plan_of(w):
    return dd.Plan(w.freqs, w.tsamp, w.nsamp, w.ranges, w.dtype)


@pytest.mark.parametrize("make", [synth.tiny, synth.ska_single_beam, synth.differentiable,
                                  lambda: synth.batched_differentiable(1)[0],
                                  lambda: synth.batched_beams(3)[2]])
def test_plan_matches_oracle_exactly(make):
    w = make()
    p = plan_of(w)
    op = O.expand_plan(w.freqs, w.tsamp, w.nsamp, w.ranges)
    assert p.ndms_total == sum(len(r.dms) for r in op)
    np.testing.assert_array_equal(p.dms(), np.concatenate([r.dms for r in op]))
    np.testing.assert_array_equal(p.shifts(), np.concatenate([r.shifts for r in op]))
    off = 0
    for ri, r in zip(p.ranges, op):
        assert (ri.ndms, ri.nout, ri.max_shift, ri.downsample) == \
            (len(r.dms), r.nout, int(r.shifts.max()), r.ds)
        assert ri.out_offset == off
        off += ri.ndms * ri.nout
    assert p.out_elems == off
    assert p.overlap == O.overlap_samples(op)
    p.close()


def test_ska_plan_sizes_and_workspace():
    w = synth.ska_single_beam()
    p = plan_of(w)
    assert p.out_elems == 536529400
    assert p.overlap == 22560
    # 16-bit copies for ds = 1, 2, 4, 8, 16 (padded rows)
    want = sum(4096 * (w.nsamp // ds) * 2 for ds in (1, 2, 4, 8, 16))
    assert want <= p.workspace_bytes < want * 1.01
    assert p.strategy["workgroups"] > 8 * 256


def test_random_plans_match_oracle():
    rng = np.random.default_rng(7)
    for _ in range(20):
        nch = int(rng.integers(1, 300))
        freqs = rng.uniform(200.0, 2000.0, nch)
        tsamp = float(rng.choice([64e-6, 1e-4, 1e-3]))
        nsamp = int(rng.integers(2000, 50000))
        ranges = []
        lo = 0.0
        for _r in range(int(rng.integers(1, 5))):
            step = float(rng.choice([0.05, 0.3, 1.0, 2.5]))
            n = int(rng.integers(1, 60))
            ranges.append((lo, lo + n * step, step, int(rng.choice([1, 2, 3, 4, 8]))))
            lo += n * step
        try:
            op = O.expand_plan(freqs, tsamp, nsamp, ranges)
        except ValueError:
            with pytest.raises(dd.DDError) as e:
                dd.Plan(freqs, tsamp, nsamp, ranges)
            assert e.value.status == -3
            continue
        p = dd.Plan(freqs, tsamp, nsamp, ranges)
        np.testing.assert_array_equal(p.shifts(), np.concatenate([r.shifts for r in op]))
        assert [r.nout for r in p.ranges] == [r.nout for r in op]


BAD = [
    (dict(nchans_override=0), -2),
    (dict(tsamp=0.0), -2),
    (dict(tsamp=float("nan")), -2),
    (dict(nsamp=0), -2),
    (dict(ranges=[]), -2),
    (dict(ranges=[(10.0, 5.0, 1.0, 1)]), -2),
    (dict(ranges=[(0.0, 5.0, 0.0, 1)]), -2),
    (dict(ranges=[(-1.0, 5.0, 1.0, 1)]), -2),
    (dict(ranges=[(0.0, 5.0, 1.0, 0)]), -2),
    (dict(ranges=[(0.0, 5.0, 1.0, 300)]), -2),
    (dict(ranges=[(0.0, 0.2, 1.0, 1)]), -2),          # rounds to zero DMs
    (dict(ranges=[(0.0, 60000.0, 100.0, 1)]), -3),   # delays exceed the data
    (dict(freq0=-1.0), -2),
    (dict(freq0=float("inf")), -2),
    (dict(ranges=[(0.0, 1.0, 1.0, 1)] * 17), -2),     # more than DD_MAX_RANGES
]


@pytest.mark.parametrize("kw,code", BAD)
def test_plan_validation_errors(kw, code):
    freqs = synth.channel_freqs(1500.0, -2.34375, 16)
    if "freq0" in kw:
        freqs = freqs.copy()
        freqs[0] = kw["freq0"]
    ranges = kw.get("ranges", [(0.0, 10.0, 1.0, 1)])
    L = _lib.lib()
    rg = (dd._Range * max(1, len(ranges)))(*[dd._Range(*r) for r in ranges])
    h = ctypes.c_void_p(1)
    st = L.dd_plan_create(freqs.ctypes.data_as(ctypes.c_void_p),
                          kw.get("nchans_override", len(freqs)), kw.get("tsamp", 1e-3),
                          kw.get("nsamp", 4096), rg, len(ranges), 0, ctypes.byref(h))
    assert st == code
    assert not h.value
    assert len(L.dd_last_error()) > 0


def test_overflow_guard():
    freqs = synth.band_freqs(1670.0, 1370.0, 600000)
    with pytest.raises(dd.DDError) as e:
        dd.Plan(freqs, 64e-6, 4096, [(0.0, 0.1, 0.1, 16)])
    assert e.value.status == -4
    # the float path has no int32 guard
    dd.Plan(freqs[:1000], 64e-6, 4096, [(0.0, 0.1, 0.1, 16)], "f32").close()


def test_null_arguments():
    L = _lib.lib()
    assert L.dd_plan_create(None, 1, 1.0, 1, None, 1, 0, None) == -1
    assert L.dd_plan_info(None, None, None, None) == -1
    assert L.dd_workspace_bytes(None, None) == -1
    assert L.dd_forward(None, None, None, None, 0, None, 0, None) == -1
    L.dd_plan_destroy(None)
    for code in range(-9, 1):
        assert L.dd_status_str(code)


def test_forward_argument_errors_precede_device_work():
    """Capacity, workspace and dtype errors are reported synchronously and
    before any HIP call (the pointers below are never dereferenced)."""
    w = synth.ska_single_beam()
    p = plan_of(w)
    L = _lib.lib()
    fake = ctypes.c_void_p(0x1000)
    st = L.dd_forward(p.handle, fake, None, fake, p.out_elems - 1, fake, p.workspace_bytes, None)
    assert st == -5
    st = L.dd_forward(p.handle, fake, None, fake, p.out_elems, fake, p.workspace_bytes - 1, None)
    assert st == -9
    st = L.dd_forward(p.handle, fake, None, fake, p.out_elems, None, p.workspace_bytes, None)
    assert st == -9
    st = L.dd_forward(p.handle, fake, fake, fake, p.out_elems, fake, p.workspace_bytes, None)
    assert st == -6
    assert b"weights" in L.dd_last_error()


def test_plan_create_destroy_many():
    w = synth.tiny()
    for _ in range(200):
        plan_of(w).close()


def test_strategy_is_queryable():
    p = plan_of(synth.tiny())
    s = p.strategy
    assert s["time_tile"] > 0 and s["dm_tile"] > 0 and s["chans_stage"] >= 1
    r = p.ranges[0]
    assert s["workgroups"] == -(-r.nout // s["time_tile"]) * -(-r.ndms // s["dm_tile"])


def test_stream_step_of_the_ska_plan():
    """The chunk step of the SKA-like plan is nsamp minus its largest delay
    in native samples (22560), a multiple of every downsample."""
    p = plan_of(synth.ska_single_beam())
    L = _lib.lib()
    h = ctypes.c_void_p()
    assert L.dd_stream_create(p.handle, 0, ctypes.byref(h)) == 0
    first, step = ctypes.c_int64(), ctypes.c_int64()
    assert L.dd_stream_info(h, ctypes.byref(first), ctypes.byref(step)) == 0
    assert first.value == 262144 and step.value == 262144 - 22560
    L.dd_stream_destroy(h)
    assert L.dd_stream_create(p.handle, 2, ctypes.byref(h)) == -2
    short = dd.Plan(synth.band_freqs(1670.0, 1370.0, 64), 64e-6, 3000, [(0.0, 150.0, 1.0, 1)])
    assert L.dd_stream_create(short.handle, 0, ctypes.byref(h)) == -2   # step < nsamp/2


def test_subband_variant_strategy():
    """Variant 3 (exact sub-band reuse) on the SKA-like plan: 192-DM tiles
    of 256 samples with 16-channel stages by default, 256-sample tiles at
    dm_tile 128, 512-sample tiles at 96 and 64; the workgroup count follows
    the tiles."""
    w = synth.ska_single_beam()
    for dm_tile, tt in ((0, 256), (192, 256), (128, 256), (96, 512), (64, 512)):
        p = dd.Plan(w.freqs, w.tsamp, w.nsamp, w.ranges, "u8", variant=3, dm_tile=dm_tile)
        s = p.strategy
        assert s["variant"] == 3 and s["time_tile"] == tt
        assert s["dm_tile"] == (dm_tile or 192)
        assert s["chans_stage"] % 8 == 0
        assert s["workgroups"] == sum(-(-r.nout // tt) * -(-r.ndms // s["dm_tile"])
                                      for r in p.ranges)
        assert p.out_elems == 536529400
        p.close()


@pytest.mark.parametrize("opts", [dict(variant=3, dm_tile=32), dict(variant=1, dm_tile=128),
                                  dict(variant=2, dm_tile=96), dict(variant=4),
                                  dict(variant=0, dm_tile=48)])
def test_subband_option_errors(opts):
    w = synth.tiny()
    with pytest.raises(dd.DDError) as e:
        dd.Plan(w.freqs, w.tsamp, w.nsamp, w.ranges, "u8", **opts)
    assert e.value.status == -2


def test_float_subband_variants_and_batches_mix_kernels():
    """For float32 plans variant 3 forces sub-band reuse (stages of 8 rows,
    reported as variant 3), variant 1 forbids it (direct sums, reported as
    variant 2 like before), and a one-channel plan cannot share patterns
    (DD_ERR_INVALID when forced).  A batch may mix integer kernels (variant
    family and DM tile): each kernel's plans form one group of work items,
    summed by their own persistent launch."""
    w = synth.tiny()
    pf3 = dd.Plan(w.freqs, w.tsamp, w.nsamp, w.ranges, "f32", variant=3)
    assert pf3.strategy["variant"] == 3 and pf3.strategy["chans_stage"] == 8
    pf1 = dd.Plan(w.freqs, w.tsamp, w.nsamp, w.ranges, "f32", variant=1)
    assert pf1.strategy["variant"] == 2
    with pytest.raises(dd.DDError) as e:
        dd.Plan(w.freqs[:1], w.tsamp, w.nsamp, w.ranges, "f32", variant=3)
    assert e.value.status == -2
    p3 = dd.Plan(w.freqs, w.tsamp, w.nsamp, w.ranges, "u8", variant=3)
    p3b = dd.Plan(w.freqs, w.tsamp, w.nsamp // 2, w.ranges, "u8", variant=3)
    p3_128 = dd.Plan(w.freqs, w.tsamp, w.nsamp, w.ranges, "u8", variant=3, dm_tile=128)
    p1 = dd.Plan(w.freqs, w.tsamp, w.nsamp, w.ranges, "u8", variant=1)
    p2 = dd.Plan(w.freqs, w.tsamp, w.nsamp, w.ranges, "u8", variant=2)

    def items(p):
        tt, dt = p.strategy["time_tile"], p.strategy["dm_tile"]
        return sum(-(-r.nout // tt) * -(-r.ndms // dt) for r in p.ranges)

    for mix in ([p3, p3b], [p1, p2], [p3, p1], [p1, p3, p3_128, p2, p3b]):
        b = dd.Batch(mix)
        assert b.work_items == sum(items(p) for p in mix)
        b.close()


def test_float_batches_layout_and_dtype_mixing():
    """A batch holds plans of one dtype.  A float32 batch lays out each
    beam's float32 input (4 bytes a sample) and output at 256-byte aligned
    offsets, forms one kernel group (variant 0, 32-output tile) whose work
    items are the forward workgroups of every beam, and sizes its workspace
    for the beams' forwards only."""
    w = synth.tiny()
    pf = [dd.Plan(w.freqs, w.tsamp, n, w.ranges, "f32") for n in (w.nsamp, w.nsamp // 2 + 3)]
    pu = dd.Plan(w.freqs, w.tsamp, w.nsamp, w.ranges, "u8")
    with pytest.raises(dd.DDError) as e:
        dd.Batch([pf[0], pu])
    assert e.value.status == -6
    b = dd.Batch(pf)
    assert b.dtype == "f32" and len(b.groups) == 1
    assert b.groups[0]["variant"] == 0 and b.groups[0]["dm_tile"] == 32
    assert b.in_offsets[0] == 0 and b.in_offsets[1] >= 4 * pf[0].nchans * pf[0].nsamp
    assert all(o % 256 == 0 for o in b.in_offsets) and all(o % 64 == 0 for o in b.out_offsets)
    assert b.in_bytes >= b.in_offsets[1] + 4 * pf[1].nchans * pf[1].nsamp
    assert b.out_elems >= b.out_offsets[1] + pf[1].out_elems
    assert b.workspace_bytes < sum(p.workspace_bytes for p in pf)
    tiles = sum(-(-r.nout // 1008) * -(-r.ndms // 32) for p in pf for r in p.ranges)
    assert b.work_items == tiles
    b.close()


def test_default_strategy_prefers_exact_subband_reuse():
    """Variant 0 (the default) takes exact sub-band reuse at 192-DM tiles
    when the plan's delay patterns fit the LDS, else 128-DM tiles, else the
    direct kernel at 64-DM tiles; and the direct kernel too when the tile
    holds more than one distinct pattern per four DMs and sub-band.  A
    requested DM tile is kept."""
    w = synth.ska_single_beam()
    s = dd.Plan(w.freqs, w.tsamp, w.nsamp, w.ranges).strategy
    assert (s["variant"], s["dm_tile"], s["time_tile"]) == (3, 192, 256)
    s = dd.Plan(w.freqs, w.tsamp, w.nsamp, w.ranges, dm_tile=96).strategy
    assert (s["variant"], s["dm_tile"], s["time_tile"]) == (3, 96, 512)
    s = dd.Plan(w.freqs, w.tsamp, w.nsamp, w.ranges, dm_tile=32).strategy
    assert (s["variant"], s["dm_tile"]) == (1, 32)
    # 1024 wide channels at 128 us, DM step 1: too many delay patterns for
    # the LDS at 192-DM tiles; they fit at 128, but with about one pattern
    # per three DMs reuse does not pay, so the default is the direct kernel
    d = synth.differentiable()
    with pytest.raises(dd.DDError):
        dd.Plan(d.freqs, d.tsamp, d.nsamp, d.ranges, "u8", variant=3)
    s = dd.Plan(d.freqs, d.tsamp, d.nsamp, d.ranges, "u8", variant=3, dm_tile=128).strategy
    assert (s["variant"], s["dm_tile"]) == (3, 128)
    p = dd.Plan(d.freqs, d.tsamp, d.nsamp, d.ranges, "u8")
    assert (p.strategy["variant"], p.strategy["dm_tile"]) == (1, 64)
    assert p.shifts().shape == (512, 1024)
    # the tiny plan (128 channels, DM step 1 at 256 us) fits at 192 but is as
    # dense, and so is a 64-channel band
    t = synth.tiny()
    assert dd.Plan(t.freqs, t.tsamp, t.nsamp, t.ranges, "u8").strategy["variant"] == 1
    assert dd.Plan(t.freqs, t.tsamp, t.nsamp, t.ranges, "u8", variant=3).strategy["variant"] == 3
    f64 = synth.band_freqs(1500.0, 1200.0, 64)
    assert dd.Plan(f64, 256e-6, 1 << 18, [(0.0, 200.0, 0.5, 1)], "u8").strategy["variant"] == 1
    # 1024 channels of the SKA-like band to DM 500: sparse patterns, reuse
    s = dd.Plan(synth.band_freqs(1670.0, 1370.0, 1024), 64e-6, 1 << 18,
                synth.ska_ranges_upto(500.0), "u8").strategy
    assert (s["variant"], s["dm_tile"]) == (3, 192)
    # DM step 2: too many at every sub-band tile, so the direct kernel
    coarse = [(0.0, 1024.0, 2.0, 1)]
    for tile in (192, 128, 96, 64):
        with pytest.raises(dd.DDError):
            dd.Plan(d.freqs, d.tsamp, d.nsamp, coarse, "u8", variant=3, dm_tile=tile)
    p = dd.Plan(d.freqs, d.tsamp, d.nsamp, coarse, "u8")
    assert (p.strategy["variant"], p.strategy["dm_tile"]) == (1, 64)
    s = dd.Plan(d.freqs, d.tsamp, d.nsamp, coarse, "u8", dm_tile=192).strategy
    assert (s["variant"], s["dm_tile"]) == (1, 64)


def test_subband_variant_rejects_plans_beyond_the_lds():
    """A DM tile whose delays spread over thousands of samples needs more
    LDS than a workgroup has: DD_ERR_INVALID at creation, naming the LDS."""
    freqs = synth.band_freqs(500.0, 300.0, 64)
    with pytest.raises(dd.DDError) as e:
        dd.Plan(freqs, 1e-3, 20000, [(0.0, 400.0, 12.5, 1)], "u8", variant=3)
    assert e.value.status == -2 and "LDS" in str(e.value)


# fixed part of an item's cost in channels (the batch's documented cost model)
ITEM_OVERHEAD_CHANS = 330.0


def _queue_costs(batch, plans, g=0):
    """Per-XCD cost (items x (their beam's channels + the fixed part)) of
    group g's queues, from the item order the batch documents: the group's
    (beam, range) lists in beam order, stably sorted by channel count, most
    first."""
    G = batch.groups[g]
    descs = []
    for p in plans:
        s = p.strategy
        if (s["variant"], s["dm_tile"]) != (G["variant"], G["dm_tile"]):
            continue
        for r in p.ranges:
            n = -(-r.nout // s["time_tile"]) * -(-r.ndms // s["dm_tile"])
            descs.append((p.nchans, n))
    descs.sort(key=lambda d: -d[0])
    weights = np.concatenate([np.full(n, c + ITEM_OVERHEAD_CHANS) for c, n in descs])
    assert len(weights) == G["work_items"]
    prefix = np.concatenate([[0], np.cumsum(weights)])
    qb = G["queue_bounds"]
    return [float(prefix[qb[x + 1]] - prefix[qb[x]]) for x in range(8)], float(prefix[-1]), weights


def test_batch_queues_share_the_cost_evenly():
    """Beams of 4096 and 1024 channels: each XCD queue holds an eighth of
    the group's cost (items weighted by channel count plus a fixed part) to
    within one item, so the queues hold unequal item counts."""
    freqs = {n: synth.band_freqs(1670.0, 1370.0, n) for n in (1024, 4096)}
    ranges = synth.ska_ranges_upto(500.0)
    plans = [dd.Plan(freqs[n], 64e-6, 1 << 16, ranges, "u8", variant=3)
             for n in (4096, 1024, 1024, 4096, 1024, 1024, 1024, 4096)]
    batch = dd.Batch(plans)
    assert len(batch.groups) == 1
    costs, total, weights = _queue_costs(batch, plans)
    qb = batch.groups[0]["queue_bounds"]
    assert qb[0] == 0 and qb[-1] == batch.work_items
    assert all(a <= b for a, b in zip(qb, qb[1:]))
    for c in costs:
        assert abs(c - total / 8) <= weights.max()
    counts = [qb[x + 1] - qb[x] for x in range(8)]
    assert max(counts) > 2 * min(counts)          # the 1024-channel items are cheaper


def test_batch_of_default_plans_groups_by_kernel():
    """Default plans whose patterns do or do not fit the LDS run different
    kernels: one group, with its own balanced queues, per kernel."""
    plans = []
    for nch, tsamp in ((256, 128e-6), (7, 64e-6), (64, 128e-6), (7, 64e-6)):
        plans.append(dd.Plan(synth.band_freqs(1670.0, 1370.0, nch), tsamp, 6000,
                             synth.ska_ranges_upto(150.0), "u8"))
    kernels = {(p.strategy["variant"], p.strategy["dm_tile"]) for p in plans}
    batch = dd.Batch(plans)
    assert {(g["variant"], g["dm_tile"]) for g in batch.groups} == kernels and len(kernels) > 1
    assert sum(g["work_items"] for g in batch.groups) == batch.work_items
    for g in range(len(batch.groups)):
        costs, total, weights = _queue_costs(batch, plans, g)
        assert abs(sum(costs) - total) <= 1e-6 * total
        assert all(abs(c - total / 8) <= weights.max() for c in costs)


def _pattern_density(plan, tile=192, K=8, max_spread=125):
    """Distinct delay patterns per real DM and 8-channel sub-band, weighted
    by each range's DM-trial samples, counted here from the plan's shift
    table: in each DM tile and sub-band, DMs whose delays minus their
    smallest delay agree share a pattern (a pattern whose smallest delays
    spread over more than max_spread samples counts again)."""
    S = plan.shifts()
    num = den = 0.0
    off = 0
    for ri in plan.ranges:
        s = S[off: off + ri.ndms]
        off += ri.ndms
        J = 0
        nsub = -(-plan.nchans // K)
        for g in range(0, ri.ndms, tile):
            blk = s[g: g + tile]
            for b in range(nsub):
                sb = blk[:, b * K: (b + 1) * K]
                a = sb.min(axis=1)
                firsts = {}
                for i in range(len(sb)):
                    key = tuple(sb[i] - a[i])
                    if key not in firsts or a[i] - firsts[key] > max_spread:
                        firsts[key] = a[i]
                        J += 1
        w = ri.ndms * ri.nout
        num += w * J / (ri.ndms * nsub)
        den += w
    return num / den


@pytest.mark.parametrize("nch,tsamp,f_top,bw,step,ndms,want", [
    # ragged last tiles (216, 198, 203 DMs at 192-DM tiles): per real DM the
    # density is above the crossover, per padded tile it would be below it
    (256, 128e-6, 1400.0, 100.0, 1.0, 216, 1),
    (64, 128e-6, 1430.0, 250.0, 0.1, 198, 1),
    (96, 64e-6, 1530.0, 54.0, 0.2, 203, 1),
    # below the crossover either way
    (256, 128e-6, 1670.0, 70.0, 1.0, 305, 3),
    (128, 128e-6, 1530.0, 250.0, 0.1, 255, 3),
])
def test_default_density_counts_real_dms(nch, tsamp, f_top, bw, step, ndms, want):
    """The default takes sub-band reuse only when a tile holds at most one
    pattern per four real DMs and sub-band: the padding DMs of a range's
    last DM tile have no sums and do not dilute the density."""
    freqs = synth.band_freqs(f_top, f_top - bw, nch)
    ranges = [(0.0, ndms * step, step, 1)]
    p3 = dd.Plan(freqs, tsamp, 1 << 16, ranges, "u8", variant=3, dm_tile=192)
    dens = _pattern_density(p3)
    assert (dens > 0.25) == (want == 1), dens
    s = dd.Plan(freqs, tsamp, 1 << 16, ranges, "u8").strategy
    assert s["variant"] == want
    if want == 3:
        assert s["dm_tile"] == 192
