"""Boxcar loss on the dedispersed output (never stored) and its gradient,
which recomputes the output tiles, against the FP64 oracle."""
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


def oracle_loss_and_grads(xs, freqs, tsamp, ranges, w, widths):
    L, gX, gw = 0.0, [], np.zeros(len(freqs))
    for x in xs:
        flat = cref.dedisperse_f32(x, freqs, tsamp, ranges, w)
        plan = O.expand_plan(freqs, tsamp, x.shape[1], ranges)
        outs, off = [], 0
        for r in plan:
            n = len(r.dms) * r.nout
            outs.append(flat[off: off + n].reshape(len(r.dms), r.nout))
            off += n
        L += O.boxcar_loss(outs, widths)
        g = O.concat(O.boxcar_loss_grad(outs, widths))
        dX, dw = cref.adjoint_f32(x, freqs, tsamp, ranges, g, w)
        gX.append(dX)
        gw += dw
    return L, gX, gw


def normwise(got, want):
    return float(np.max(np.abs(got - want)) / max(np.max(np.abs(want)), 1e-30))


@pytest.mark.parametrize("seed,max_width", [(0, 32), (1, 8), (2, 1)])
def test_small_plans_vs_oracle(seed, max_width):
    rng = np.random.default_rng(900 + seed)
    nch, nsamp, nb = int(rng.integers(3, 90)), int(rng.integers(1500, 5000)), 2
    freqs = synth.band_freqs(1500.0, 1300.0, nch)
    ranges = [(0.0, 20.0, 1.0, 1), (20.0, 30.0, 2.0, 2)]
    tsamp = 2.56e-4
    xs = rng.standard_normal((nb, nch, nsamp)).astype(np.float32)
    w = rng.uniform(0.5, 1.5, nch).astype(np.float32)
    widths = tuple(2 ** i for i in range(int(np.log2(max_width)) + 1))
    say("boxcar small", seed, nch, nsamp, widths)
    plan = dd.Plan(freqs, tsamp, nsamp, ranges, "f32")
    xt, wt = torch.from_numpy(xs).cuda(), torch.from_numpy(w).cuda()
    loss = float(dd.boxcar_loss(xt, plan, wt, max_width))
    dx, dw = dd.boxcar_backward(xt, plan, wt, max_width)
    torch.cuda.synchronize()
    L, gX, gw = oracle_loss_and_grads(list(xs), freqs, tsamp, ranges, w, widths)
    assert abs(loss - L) <= 1e-5 * L
    for b in range(nb):
        assert normwise(dx[b].cpu().numpy(), gX[b]) <= 1e-5
    assert normwise(dw.cpu().numpy(), gw) <= 1e-5


def test_differentiable_beam_plan_reduced_length_vs_oracle():
    """The batched-differentiable plan (4096 channels, DM 0..999) on two
    beams shortened to 2^14 samples, against the FP64 oracle."""
    full = synth.batched_differentiable(2, nsamp=1 << 14)
    w0 = full[0]
    say("boxcar 4096ch reduced length")
    xs = [synth.filterbank_f32(w.seed, w.nchans, w.nsamp) for w in full]
    wts = (1.0 + 0.1 * synth.gaussian(7, (w0.nchans,), "weights")).astype(np.float32)
    plan = dd.Plan(w0.freqs, w0.tsamp, w0.nsamp, w0.ranges, "f32")
    xt = torch.from_numpy(np.stack(xs)).cuda()
    wt = torch.from_numpy(wts).cuda()
    loss = float(dd.boxcar_loss(xt, plan, wt))
    dx, dw = dd.boxcar_backward(xt, plan, wt)
    torch.cuda.synchronize()
    L, gX, gw = oracle_loss_and_grads(xs, w0.freqs, w0.tsamp, w0.ranges, wts, O.BOXCAR_WIDTHS)
    assert abs(loss - L) <= 1e-5 * L
    for b in range(2):
        assert normwise(dx[b].cpu().numpy(), gX[b]) <= 1e-5
    assert normwise(dw.cpu().numpy(), gw) <= 1e-5


def test_batched_differentiable_full_size():
    """32 beams x 4096 channels x 2^17 float32, DM 0..999: the loss of the
    batch is the sum of the beams' losses, the weight gradient adds over
    beams, and (the loss being quadratic in the weights) central differences
    match the weight gradient."""
    wls = synth.batched_differentiable()
    w0 = wls[0]
    say("boxcar full size: inputs")
    plan = dd.Plan(w0.freqs, w0.tsamp, w0.nsamp, w0.ranges, "f32")
    x = torch.empty((len(wls), w0.nchans, w0.nsamp), dtype=torch.float32, device="cuda")
    gen = torch.Generator(device="cuda")
    for b, w in enumerate(wls):
        gen.manual_seed(w.seed)
        x[b].normal_(generator=gen)
    wt = torch.ones(w0.nchans, dtype=torch.float32, device="cuda")
    ws = dd.workspace(plan)
    say("boxcar full size: loss + backward")
    loss = float(dd.boxcar_loss(x, plan, wt, ws=ws))
    dx, dw = dd.boxcar_backward(x, plan, wt, ws=ws)
    torch.cuda.synchronize()
    assert np.isfinite(loss) and loss > 0
    assert torch.isfinite(dx).all() and torch.isfinite(dw).all()
    per = [float(dd.boxcar_loss(x[b], plan, wt, ws=ws)) for b in range(len(wls))]
    assert abs(loss - sum(per)) <= 1e-5 * loss
    del dx
    _, dw01 = dd.boxcar_backward(x[:2], plan, wt, ws=ws, grad_in=False)
    _, dw0 = dd.boxcar_backward(x[:1], plan, wt, ws=ws, grad_in=False)
    _, dw1 = dd.boxcar_backward(x[1:2], plan, wt, ws=ws, grad_in=False)
    torch.cuda.synchronize()
    assert torch.allclose(dw01, dw0 + dw1, rtol=1e-5, atol=1e-3 * float(dw01.abs().max()) * 1e-3)
    # L(w) on one beam is a quadratic form in w: central differences are exact
    # up to rounding; the float32 loss limits agreement to ~1e-3 relative.
    h = 0.25
    for c in (0, 2048, 4095):
        e = torch.zeros_like(wt)
        e[c] = h
        lp = float(dd.boxcar_loss(x[0], plan, wt + e, ws=ws))
        lm = float(dd.boxcar_loss(x[0], plan, wt - e, ws=ws))
        fd = (lp - lm) / (2 * h)
        assert abs(fd - float(dw0[c])) <= 2e-3 * abs(float(dw0[c])) + 1e-6 * lp, (c, fd, float(dw0[c]))


@pytest.mark.timeout(1200)
def test_differentiable_beam_full_length_vs_oracle():
    """One whole beam of the batched-differentiable workload (4096 channels
    x 2^17 float32 samples, DM 0..999, widths 1..32, non-unit weights)
    against the FP64 oracle: the loss, dL/dw over all channels and dL/dx
    over the whole input."""
    w0 = synth.batched_differentiable(1)[0]
    say("boxcar full-length beam: input", w0.nchans, w0.nsamp)
    x = synth.filterbank_f32(w0.seed, w0.nchans, w0.nsamp)
    wts = (1.0 + 0.1 * synth.gaussian(7, (w0.nchans,), "weights")).astype(np.float32)
    plan = dd.Plan(w0.freqs, w0.tsamp, w0.nsamp, w0.ranges, "f32")
    xt, wt = torch.from_numpy(x).cuda(), torch.from_numpy(wts).cuda()
    say("boxcar full-length beam: GPU loss + backward")
    loss = float(dd.boxcar_loss(xt, plan, wt))
    dx, dw = dd.boxcar_backward(xt, plan, wt)
    torch.cuda.synchronize()
    dx, dw = dx.cpu().numpy(), dw.cpu().numpy()
    del xt
    say("boxcar full-length beam: oracle forward on", cref.max_threads(), "threads")
    L, gX, gw = oracle_loss_and_grads([x], w0.freqs, w0.tsamp, w0.ranges, wts, O.BOXCAR_WIDTHS)
    rel_loss = abs(loss - L) / L
    nx, nw = normwise(dx, gX[0]), normwise(dw, gw)
    say(f"boxcar full-length beam: loss rel {rel_loss:.2e}, dx normwise {nx:.2e}, "
        f"dw normwise {nw:.2e}")
    assert rel_loss <= 1e-5
    assert nx <= 1e-5
    assert nw <= 1e-5


def test_boxcar_loss_autograd_vs_oracle():
    """The boxcar loss as a torch.autograd.Function: .backward() fills
    x.grad and w.grad with the oracle's gradients (the output recomputed,
    never saved), and an upstream scale multiplies them."""
    rng = np.random.default_rng(950)
    nch, nsamp, nb = 48, 3000, 2
    freqs = synth.band_freqs(1500.0, 1300.0, nch)
    ranges = [(0.0, 20.0, 1.0, 1), (20.0, 30.0, 2.0, 2)]
    tsamp = 2.56e-4
    xs = rng.standard_normal((nb, nch, nsamp)).astype(np.float32)
    w = rng.uniform(0.5, 1.5, nch).astype(np.float32)
    say("boxcar autograd", nch, nsamp)
    plan = dd.Plan(freqs, tsamp, nsamp, ranges, "f32")
    L, gX, gw = oracle_loss_and_grads(list(xs), freqs, tsamp, ranges, w, O.BOXCAR_WIDTHS)
    for scale in (1.0, 3.0):
        xt = torch.from_numpy(xs).cuda().requires_grad_(True)
        wt = torch.from_numpy(w).cuda().requires_grad_(True)
        loss = dd.boxcar_loss_autograd(xt, wt, plan, 32)
        (scale * loss).backward()
        torch.cuda.synchronize()
        assert abs(float(loss) - L) <= 1e-5 * L
        for b in range(nb):
            assert normwise(xt.grad[b].cpu().numpy(), scale * gX[b]) <= 1e-5
        assert normwise(wt.grad.cpu().numpy(), scale * gw) <= 1e-5
    # gradient to x only
    xt = torch.from_numpy(xs).cuda().requires_grad_(True)
    dd.boxcar_loss_autograd(xt, None, plan, 32).backward()
    L1, gX1, _ = oracle_loss_and_grads(list(xs), freqs, tsamp, ranges, np.ones(nch, np.float32),
                                       O.BOXCAR_WIDTHS)
    torch.cuda.synchronize()
    assert normwise(xt.grad[0].cpu().numpy(), gX1[0]) <= 1e-5


def uneven_float_beams(seed, n, multi_range=False):
    """Float32 beams of uneven channel counts and lengths, one full-resolution
    range each (or, with multi_range, a second downsampled range on odd beams),
    random channel weights."""
    rng = np.random.default_rng(1300 + seed)
    beams = []
    for b in range(n):
        nch = int(rng.choice([9, 40, 70]))
        nsamp = int(rng.integers(2500, 6000))
        freqs = synth.band_freqs(1500.0, float(rng.uniform(1250.0, 1400.0)), nch)
        ranges = [(0.0, float(rng.integers(8, 30)), 1.0, 1)]
        if multi_range and b % 2:
            ranges.append((ranges[0][1], ranges[0][1] + 10.0, 2.0, 2))
        x = rng.standard_normal((nch, nsamp)).astype(np.float32)
        w = rng.uniform(0.5, 1.5, nch).astype(np.float32)
        beams.append((x, freqs, 2.56e-4, ranges, w))
    return beams


@pytest.mark.parametrize("max_width", [32, 4])
def test_batch_boxcar_matches_single_plans_and_oracle(max_width):
    """The batched boxcar loss and backward (one launch per phase over every
    beam) equal each beam's own dd_boxcar_loss / dd_boxcar_backward bit for
    bit (the same partial sums in the same order) and the FP64 oracle within
    the float32 tolerance."""
    beams = uneven_float_beams(0, 5)
    widths = tuple(2 ** i for i in range(int(np.log2(max_width)) + 1))
    say("batch boxcar", max_width, [b[0].shape for b in beams])
    plans = [dd.Plan(f, t, x.shape[1], r, "f32") for (x, f, t, r, _) in beams]
    batch = dd.Batch(plans)
    xin = batch.pack([b[0] for b in beams])
    wts = batch.pack_weights([b[4] for b in beams])
    losses = dd.batch_boxcar_loss(xin, batch, wts, max_width)
    dx, dw = dd.batch_boxcar_backward(xin, batch, wts, max_width)
    torch.cuda.synchronize()
    for i, ((x, f, t, r, w), p) in enumerate(zip(beams, plans)):
        xt, wt = torch.from_numpy(x).cuda(), torch.from_numpy(w).cuda()
        l1 = dd.boxcar_loss(xt, p, wt, max_width)
        dx1, dw1 = dd.boxcar_backward(xt, p, wt, max_width)
        torch.cuda.synchronize()
        assert float(losses[i]) == float(l1), i
        assert torch.equal(batch.split_input(dx)[i], dx1), i
        assert torch.equal(batch.split_weights(dw)[i], dw1), i
        L, gX, gw = oracle_loss_and_grads([x], f, t, r, w, widths)
        assert abs(float(losses[i]) - L) <= 1e-5 * L
        assert normwise(dx1.cpu().numpy().astype(np.float64), gX[0]) <= 1e-5
        assert normwise(dw1.cpu().numpy().astype(np.float64), gw) <= 1e-5


def test_batch_boxcar_graph_replay_and_limits():
    """The batched boxcar loss and backward replay from a HIP graph (the
    workspace scribbled and eager work between replays); a multi-range plan
    batch computes the loss but refuses the batched backward."""
    beams = uneven_float_beams(1, 3)
    plans = [dd.Plan(f, t, x.shape[1], r, "f32") for (x, f, t, r, _) in beams]
    batch = dd.Batch(plans)
    batch.prepare()
    xin = batch.pack([b[0] for b in beams])
    wts = batch.pack_weights([b[4] for b in beams])
    ws = dd.batch_boxcar_workspace(batch)
    e_loss = dd.batch_boxcar_loss(xin, batch, wts, 16, ws=ws).clone()
    e_dx, e_dw = dd.batch_boxcar_backward(xin, batch, wts, 16, ws=ws)
    loss = torch.zeros(len(plans), dtype=torch.float32, device="cuda")
    dx = torch.zeros_like(e_dx)
    dw = torch.zeros_like(e_dw)
    L = dd.lib()

    def run():
        dd.check(L.dd_batch_boxcar_loss(batch.handle, dd._ptr(xin), dd._ptr(wts), 16, dd._ptr(loss),
                                        dd._ptr(ws), ws.numel(), dd._stream_ptr(None)), "loss")
        dd.check(L.dd_batch_boxcar_backward(batch.handle, dd._ptr(xin), dd._ptr(wts), 16, dd._ptr(dx),
                                            dd._ptr(dw), dd._ptr(ws), ws.numel(), dd._stream_ptr(None)),
                 "backward")

    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        run()
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        run()
    for i in range(3):
        loss.zero_()
        dx.zero_()
        dw.zero_()
        ws.fill_(0x7F)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(loss, e_loss) and torch.equal(dw, e_dw), i
        assert all(torch.equal(a, b) for a, b in zip(batch.split_input(dx), batch.split_input(e_dx))), i
        other = dd.batch_boxcar_loss(xin, batch, wts, 16)       # eager work between replays
        torch.cuda.synchronize()
        assert torch.equal(other, e_loss)
    mbeams = uneven_float_beams(2, 3, multi_range=True)
    mplans = [dd.Plan(f, t, x.shape[1], r, "f32") for (x, f, t, r, _) in mbeams]
    mb = dd.Batch(mplans)
    mx = mb.pack([b[0] for b in mbeams])
    ml = dd.batch_boxcar_loss(mx, mb, None, 8)
    torch.cuda.synchronize()
    for i, ((x, f, t, r, _), p) in enumerate(zip(mbeams, mplans)):
        assert float(ml[i]) == float(dd.boxcar_loss(torch.from_numpy(x).cuda(), p, None, 8))
    with pytest.raises(dd.DDError) as e:
        dd.batch_boxcar_backward(mx, mb, None, 8)
    assert e.value.status == -2


def test_many_tiny_float_beams_batch():
    """120 tiny float32 beams (1 to 17 channels) in one batch: the forward,
    the boxcar loss and its backward equal each beam's own calls bit for bit
    (descriptor search over many short problems; the helper launches loop
    over their descriptors)."""
    rng = np.random.default_rng(777)
    beams = []
    for b in range(120):
        nch = int(rng.choice([1, 3, 8, 17]))
        nsamp = int(rng.integers(1200, 3000))
        freqs = synth.band_freqs(1500.0, float(rng.uniform(1250.0, 1450.0)), nch)
        ranges = [(0.0, float(rng.integers(2, 20)), 1.0, 1)]
        x = rng.standard_normal((nch, nsamp)).astype(np.float32)
        w = rng.uniform(0.5, 1.5, nch).astype(np.float32)
        beams.append((x, freqs, 2.56e-4, ranges, w))
    say("many tiny float beams", len(beams))
    plans = [dd.Plan(f, t, x.shape[1], r, "f32") for (x, f, t, r, _) in beams]
    batch = dd.Batch(plans)
    xin = batch.pack([b[0] for b in beams])
    wts = batch.pack_weights([b[4] for b in beams])
    out = dd.dedisperse_batch(xin, batch, weights=wts)
    losses = dd.batch_boxcar_loss(xin, batch, wts, 8)
    dx, dw = dd.batch_boxcar_backward(xin, batch, wts, 8)
    torch.cuda.synchronize()
    for i, ((x, f, t, r, w), p, o) in enumerate(zip(beams, plans, batch.split(out))):
        xt, wt = torch.from_numpy(x).cuda(), torch.from_numpy(w).cuda()
        single = dd.dedisperse(xt, p, weights=wt)
        l1 = dd.boxcar_loss(xt, p, wt, 8)
        dx1, dw1 = dd.boxcar_backward(xt, p, wt, 8)
        torch.cuda.synchronize()
        assert torch.equal(o, single), i
        assert float(losses[i]) == float(l1), i
        assert torch.equal(batch.split_input(dx)[i], dx1), i
        assert torch.equal(batch.split_weights(dw)[i], dw1), i
