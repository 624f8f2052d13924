"""Batched forward: integer batches by persistent launches (one per kernel)
over many beams of uneven shape (direct kernel, variant 3 or both),
bit-exact against each beam's own forward and the oracle; float32 batches by
one shift-and-sum launch, bit-identical to each beam's own forward and within
the float32 tolerance of the FP64 oracle; both replayable from a HIP graph."""
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


def small_beams(seed, n, subband=False):
    """Beams of uneven shape.  For variant 3, shapes whose delay patterns fit
    the LDS at every DM tile (no 7-channel band, 128 us sampling)."""
    rng = np.random.default_rng(700 + seed)
    beams = []
    for b in range(n):
        nch = int(rng.choice([64, 130, 256] if subband else [7, 64, 130, 256]))
        nsamp = int(rng.integers(3000, 20000))
        tsamp = float(rng.choice([128e-6] if subband else [64e-6, 128e-6]))
        dm_max = float(rng.choice([150.0, 300.0, 500.0]))
        freqs = synth.band_freqs(1670.0, 1370.0, nch)
        beams.append((rng.integers(0, 256, size=(nch, nsamp)).astype(np.uint8), freqs, tsamp,
                      synth.ska_ranges_upto(dm_max)))
    return beams


# the library default (each plan's own choice: beams of one batch may run
# different kernels, one persistent launch per kernel), the direct kernel,
# and variant 3 at each of its workgroup shapes
STRATEGIES = {"auto": {}, "direct": {"variant": 1}, "v3-192": {"variant": 3},
              "v3-128": {"variant": 3, "dm_tile": 128}, "v3-96": {"variant": 3, "dm_tile": 96},
              "direct-t256": {"variant": 1, "time_tile": 256},
              "v3-64-t256": {"variant": 3, "dm_tile": 64, "time_tile": 256}}


def make_plans(beams, opts):
    return [dd.Plan(f, t, x.shape[1], r, **opts) for (x, f, t, r) in beams]


@pytest.mark.parametrize("strategy", sorted(STRATEGIES))
def test_small_batch_matches_single_plans_and_oracle(strategy):
    beams = small_beams(0, 7, strategy.startswith("v3"))
    say("small batch", strategy, [b[0].shape for b in beams])
    plans = make_plans(beams, STRATEGIES[strategy])
    batch = dd.Batch(plans)
    xin = batch.pack([b[0] for b in beams])
    out = dd.dedisperse_batch(xin, batch)
    torch.cuda.synchronize()
    for (x, f, t, r), p, o in zip(beams, plans, batch.split(out)):
        single = dd.dedisperse(torch.from_numpy(x).cuda(), p)
        torch.cuda.synchronize()
        assert torch.equal(o, single)
        assert np.array_equal(o.cpu().numpy(), cref.dedisperse_u8(x, f, t, r))


@pytest.mark.parametrize("strategy", ["auto", "direct", "v3-192"])
def test_batch_graph_replay(strategy):
    beams = small_beams(1, 5, strategy.startswith("v3"))
    say("graph replay", strategy)
    plans = make_plans(beams, STRATEGIES[strategy])
    batch = dd.Batch(plans)
    batch.prepare()
    xin = batch.pack([b[0] for b in beams])
    ws = torch.empty(batch.workspace_bytes, dtype=torch.uint8, device="cuda")
    eager = dd.dedisperse_batch(xin, batch, ws=ws).clone()
    torch.cuda.synchronize()
    want = [cref.dedisperse_u8(x, f, t, r) for (x, f, t, r) in beams]
    assert [int((o.cpu().numpy() != w).sum()) for o, w in zip(batch.split(eager), want)] == \
        [0] * len(beams), "eager batch differs from the oracle"
    out = torch.zeros(batch.out_elems, dtype=torch.int32, device="cuda")
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        dd.dedisperse_batch(xin, batch, out=out, ws=ws)        # warm-up on the capture stream
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        dd.dedisperse_batch(xin, batch, out=out, ws=ws)
    for i in range(4):
        out.zero_()
        ws.fill_(0xA5)                                        # the graph must not rely on ws contents
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        # compare the beams' outputs (the alignment gaps between beams are
        # never written)
        bad = [(int((o != e).sum()), int(((o != e) & (o == 0)).sum()))
               for o, e in zip(batch.split(out), batch.split(eager))]
        assert all(b == (0, 0) for b in bad), f"replay {i}: (mismatches, of them zeros) {bad}"
        other = dd.dedisperse(torch.from_numpy(beams[0][0]).cuda(), plans[0])   # eager work between
        torch.cuda.synchronize()
        assert torch.equal(other, batch.split(eager)[0])


@pytest.mark.parametrize("strategy", ["direct", "v3-192"])
def test_batched_beams_full_size(strategy):
    """The 64-beam batched workload (channel counts 1024/2048/4096, lengths
    2^16..2^18, DM max 500/1000/2000), drawn on the GPU: every beam of the
    batch equals its own dd_forward, one whole beam of each channel count
    equals the C oracle, and sampled outputs of three beams equal the numpy
    oracle."""
    wls = synth.batched_beams()
    say("batched beams: plans", strategy)
    plans = [dd.Plan(w.freqs, w.tsamp, w.nsamp, w.ranges, **STRATEGIES[strategy]) for w in wls]
    batch = dd.Batch(plans)
    say("batched beams: inputs", batch.in_bytes, batch.out_elems, batch.workspace_bytes)
    xin = torch.empty(batch.in_bytes, dtype=torch.uint8, device="cuda")
    for w, p, off in zip(wls, plans, batch.in_offsets):
        xin[off: off + p.nchans * p.nsamp] = synth.filterbank_u8_device(
            w.seed, w.freqs, w.tsamp, w.nsamp, w.pulses).reshape(-1)
    say("batched beams: forward")
    out = dd.dedisperse_batch(xin, batch)
    torch.cuda.synchronize()
    outs = batch.split(out)
    ws = dd.workspace(max(plans, key=lambda q: q.workspace_bytes))
    for i, (w, p, off) in enumerate(zip(wls, plans, batch.in_offsets)):
        x = xin[off: off + p.nchans * p.nsamp].view(p.nchans, p.nsamp)
        single = torch.empty(p.out_elems, dtype=torch.int32, device="cuda")
        dd.dedisperse(x, p, out=single, ws=ws[: p.workspace_bytes] if p.workspace_bytes else None)
        torch.cuda.synchronize()
        assert torch.equal(outs[i], single), f"beam {i}"
    del ws
    # whole outputs against the C oracle: for each channel count, the beam
    # with the most DM trials (ties: the longest)
    for nch in sorted({p.nchans for p in plans}):
        i = max((j for j, p in enumerate(plans) if p.nchans == nch),
                key=lambda j: (plans[j].ndms_total, plans[j].nsamp))
        w, p, off = wls[i], plans[i], batch.in_offsets[i]
        say("batched beams: whole output of beam", i, nch, p.nsamp, p.ndms_total)
        x = xin[off: off + p.nchans * p.nsamp].view(p.nchans, p.nsamp).cpu().numpy()
        want = cref.dedisperse_u8(x, w.freqs, w.tsamp, w.ranges)
        assert np.array_equal(outs[i].cpu().numpy(), want), f"beam {i} vs oracle"
    rng = np.random.default_rng(3)
    for i in sorted({0, len(wls) - 1, int(rng.integers(len(wls)))}):
        w, p, off = wls[i], plans[i], batch.in_offsets[i]
        x = xin[off: off + p.nchans * p.nsamp].view(p.nchans, p.nsamp).cpu().numpy()
        op = O.expand_plan(w.freqs, w.tsamp, w.nsamp, w.ranges)
        per = p.split(outs[i])
        say("batched beams: oracle samples of beam", i)
        for r, ri in enumerate(p.ranges):
            d = rng.integers(0, ri.ndms, 40)
            t = rng.integers(0, ri.nout, 40)
            got = per[r][torch.from_numpy(d).cuda(), torch.from_numpy(t).cuda()].cpu().numpy()
            assert np.array_equal(got, O.dedisperse_at(x, op, r, d, t))


def float_beams(seed, n):
    """Float32 beams of uneven shape: channel counts, lengths, sampling, and
    one to three ranges with downsampling, random channel weights."""
    rng = np.random.default_rng(900 + seed)
    beams = []
    for b in range(n):
        nch = int(rng.choice([7, 33, 64, 130]))
        nsamp = int(rng.integers(2500, 9000))
        tsamp = float(rng.choice([64e-6, 128e-6, 2.56e-4]))
        freqs = synth.band_freqs(1500.0, float(rng.uniform(1200.0, 1450.0)), nch)
        ranges = [(0.0, float(rng.integers(5, 60)), 1.0, 1)]
        if b % 2:
            ranges.append((ranges[0][1], ranges[0][1] + 20.0, 2.0, int(rng.choice([2, 3]))))
        x = rng.standard_normal((nch, nsamp)).astype(np.float32)
        w = rng.uniform(0.25, 2.0, nch).astype(np.float32)
        beams.append((x, freqs, tsamp, ranges, w))
    return beams


def float_close(got, want, terms, what):
    """Float32 against the FP64 oracle: 1e-5 normwise and elementwise
    1e-5 * sum of |terms| (the float32 tolerance)."""
    got = got.astype(np.float64)
    err = np.abs(got - want)
    assert err.max() <= 1e-5 * max(np.abs(want).max(), 1e-30), what
    assert (err <= 1e-5 * terms + 1e-30).all(), what


def test_float_batch_matches_single_plans_and_oracle():
    """One shift-and-sum launch over every (beam, range) of a float32 batch
    equals each beam's own weighted forward bit for bit (the same sums in
    the same order) and the FP64 oracle within the float32 tolerance; the
    unweighted call equals unit weights."""
    beams = float_beams(0, 6)
    say("float batch", [(x.shape, len(r)) for (x, _, _, r, _) in beams])
    plans = [dd.Plan(f, t, x.shape[1], r, "f32") for (x, f, t, r, _) in beams]
    batch = dd.Batch(plans)
    xin = batch.pack([b[0] for b in beams])
    wts = batch.pack_weights([b[4] for b in beams])
    out = dd.dedisperse_batch(xin, batch, weights=wts)
    unit = dd.dedisperse_batch(xin, batch)
    ones = dd.dedisperse_batch(xin, batch, weights=torch.ones_like(wts))
    torch.cuda.synchronize()
    # per beam: the alignment gaps between beams are never written
    assert all(torch.equal(u, o) for u, o in zip(batch.split(unit), batch.split(ones)))
    for (x, f, t, r, w), p, o in zip(beams, plans, batch.split(out)):
        single = dd.dedisperse(torch.from_numpy(x).cuda(), p, weights=torch.from_numpy(w).cuda())
        torch.cuda.synchronize()
        assert torch.equal(o, single)
        want = cref.dedisperse_f32(x, f, t, r, w)
        terms = cref.dedisperse_f32(np.abs(x), f, t, r, np.abs(w))
        float_close(o.cpu().numpy(), want, terms, f"beam {x.shape}")


def test_float_batch_graph_replay():
    """The float32 batch's launches replay from a HIP graph, with the
    workspace scribbled and eager work between replays."""
    beams = float_beams(1, 4)
    say("float batch graph replay")
    plans = [dd.Plan(f, t, x.shape[1], r, "f32") for (x, f, t, r, _) in beams]
    batch = dd.Batch(plans)
    batch.prepare()
    xin = batch.pack([b[0] for b in beams])
    wts = batch.pack_weights([b[4] for b in beams])
    ws = torch.empty(batch.workspace_bytes, dtype=torch.uint8, device="cuda")
    eager = dd.dedisperse_batch(xin, batch, ws=ws, weights=wts).clone()
    out = torch.zeros(batch.out_elems, dtype=torch.float32, device="cuda")
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        dd.dedisperse_batch(xin, batch, out=out, ws=ws, weights=wts)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        dd.dedisperse_batch(xin, batch, out=out, ws=ws, weights=wts)
    for i in range(3):
        out.zero_()
        ws.fill_(0x7F)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for o, e in zip(batch.split(out), batch.split(eager)):
            assert torch.equal(o, e), f"replay {i}"
        other = dd.dedisperse(torch.from_numpy(beams[0][0]).cuda(), plans[0],
                              weights=torch.from_numpy(beams[0][4]).cuda())
        torch.cuda.synchronize()
        assert torch.equal(other, batch.split(eager)[0])


def test_many_tiny_beams():
    """200 tiny integer beams (1 to 17 channels, one or two ranges) in one
    batch of default plans: every beam equals its own forward bit for bit
    (descriptor search, queue slices and work stealing over many short
    items)."""
    rng = np.random.default_rng(4242)
    beams = []
    for b in range(200):
        nch = int(rng.choice([1, 3, 8, 17]))
        nsamp = int(rng.integers(800, 3000))
        freqs = synth.band_freqs(1500.0, float(rng.uniform(1250.0, 1450.0)), nch)
        ranges = [(0.0, float(rng.integers(2, 30)), 1.0, 1)]
        if b % 3 == 1:
            ranges.append((ranges[0][1], ranges[0][1] + 10.0, 2.0, int(rng.choice([2, 4]))))
        beams.append((rng.integers(0, 256, size=(nch, nsamp)).astype(np.uint8), freqs, 2.56e-4, ranges))
    say("many tiny beams", len(beams))
    plans = make_plans(beams, {})
    batch = dd.Batch(plans)
    xin = batch.pack([b[0] for b in beams])
    out = dd.dedisperse_batch(xin, batch)
    torch.cuda.synchronize()
    for i, ((x, f, t, r), p, o) in enumerate(zip(beams, plans, batch.split(out))):
        single = dd.dedisperse(torch.from_numpy(x).cuda(), p)
        torch.cuda.synchronize()
        assert torch.equal(o, single), i
        if i % 25 == 0:
            assert np.array_equal(o.cpu().numpy(), cref.dedisperse_u8(x, f, t, r)), i
