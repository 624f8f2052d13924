"""Float32 forward with per-channel weights, its hand-written adjoint, and
the autograd wrapper, against the FP64 oracle.

Tolerance (from the float32 reading of "rel. error <= 1e-5"): normwise
||y - y64||_inf / ||y64||_inf <= 1e-5 per output tensor, and elementwise
|y - y64| <= 1e-5 * sum|terms| + tiny.  Every call goes through the C ABI.
"""
import numpy as np
import pytest

import synth
from oracle import cref
from oracle import dedisp as O

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
dd = pytest.importorskip("paper_1912_07704_amd")

RTOL = 1e-5


def say(*a):
    print("[case]", *a, flush=True)


def normwise(got, want):
    return float(np.max(np.abs(got - want)) / max(np.max(np.abs(want)), 1e-30))


def check_close(got, want, terms_abs, what):
    nw = normwise(got, want)
    assert nw <= RTOL, f"{what}: normwise {nw:.3e}"
    bad = np.abs(got - want) > RTOL * terms_abs + 1e-30
    assert not bad.any(), f"{what}: {int(bad.sum())} elements outside the elementwise bound"


def case(seed, nch=None, nsamp=None, ranges=None):
    rng = np.random.default_rng(500 + seed)
    nch = nch or int(rng.integers(1, 200))
    nsamp = nsamp or int(rng.integers(600, 6000))
    freqs = synth.band_freqs(1500.0, float(rng.uniform(1150.0, 1450.0)), nch)
    if seed % 2:
        freqs = rng.permutation(freqs)
    ranges = ranges or [(0.0, float(rng.integers(1, 40)), 1.0, 1),
                        (40.0, 60.0, 2.0, int(rng.choice([2, 3, 4])))]
    x = rng.standard_normal((nch, nsamp)).astype(np.float32)
    w = rng.uniform(0.25, 2.0, nch).astype(np.float32)
    return x, freqs, 2.56e-4, ranges, w


def gpu_plan(freqs, tsamp, nsamp, ranges):
    return dd.Plan(freqs, tsamp, nsamp, ranges, "f32")


@pytest.mark.parametrize("seed", range(6))
def test_forward_random_shapes(seed):
    x, freqs, tsamp, ranges, w = case(seed)
    try:
        O.expand_plan(freqs, tsamp, x.shape[1], ranges)
    except ValueError:
        pytest.skip("plan has no valid output")
    say("f32 forward", seed, x.shape, ranges)
    plan = gpu_plan(freqs, tsamp, x.shape[1], ranges)
    out = dd.dedisperse(torch.from_numpy(x).cuda(), plan, weights=torch.from_numpy(w).cuda())
    torch.cuda.synchronize()
    want = cref.dedisperse_f32(x, freqs, tsamp, ranges, w)
    terms = cref.dedisperse_f32(np.abs(x), freqs, tsamp, ranges, np.abs(w))
    check_close(out.cpu().numpy().astype(np.float64), want, terms, "forward")


@pytest.mark.parametrize("variant", [1, 3])
@pytest.mark.parametrize("seed", range(8))
def test_direct_and_subband_sums_vs_oracle(seed, variant):
    """The two float32 strategies -- direct sums (variant 1) and sub-band
    reuse (variant 3: pattern rows of 4-row groups built in LDS, added at
    each output's offset) -- forward and adjoint against the FP64 oracle."""
    x, freqs, tsamp, ranges, w = case(200 + seed, nch=int(np.random.default_rng(seed).integers(9, 160)))
    try:
        O.expand_plan(freqs, tsamp, x.shape[1], ranges)
    except ValueError:
        pytest.skip("plan has no valid output")
    say("f32 variant", variant, seed, x.shape, ranges)
    try:
        plan = dd.Plan(freqs, tsamp, x.shape[1], ranges, "f32", variant=variant)
    except dd.DDError as e:
        # sub-band reuse asked for where its tables exceed the LDS is refused
        # at plan creation (the default then takes the direct sums)
        if variant == 3 and e.status == -2:
            pytest.skip(f"sub-band tables do not fit the LDS: {e}")
        raise
    assert plan.strategy["variant"] == (3 if variant == 3 else 2)
    xt, wt = torch.from_numpy(x).cuda(), torch.from_numpy(w).cuda()
    out = dd.dedisperse(xt, plan, weights=wt)
    rng = np.random.default_rng(300 + seed)
    g = rng.standard_normal(plan.out_elems).astype(np.float32)
    dx, dw = dd.adjoint(torch.from_numpy(g).cuda(), plan, x=xt, weights=wt)
    torch.cuda.synchronize()
    want = cref.dedisperse_f32(x, freqs, tsamp, ranges, w)
    terms = cref.dedisperse_f32(np.abs(x), freqs, tsamp, ranges, np.abs(w))
    check_close(out.cpu().numpy().astype(np.float64), want, terms, "forward")
    wX, ww = cref.adjoint_f32(x, freqs, tsamp, ranges, g.astype(np.float64), w)
    tX, tw = cref.adjoint_f32(np.abs(x), freqs, tsamp, ranges, np.abs(g).astype(np.float64), np.abs(w))
    check_close(dx.cpu().numpy().astype(np.float64), wX, tX, "dX")
    check_close(dw.cpu().numpy().astype(np.float64), ww, tw, "dw")


def test_forward_without_weights_equals_unit_weights():
    x, freqs, tsamp, ranges, _ = case(11, nch=33, nsamp=3000)
    say("f32 unit weights")
    plan = gpu_plan(freqs, tsamp, x.shape[1], ranges)
    xt = torch.from_numpy(x).cuda()
    a = dd.dedisperse(xt, plan)
    b = dd.dedisperse(xt, plan, weights=torch.ones(33, device="cuda"))
    torch.cuda.synchronize()
    assert torch.equal(a, b)


def test_integer_valued_float_input_is_exact():
    """uint8 values cast to float32 sum exactly (partial sums < 2^24), so the
    float path reproduces the integer path bit for bit."""
    w = synth.tiny()
    x = w.make_input()
    say("f32 on uint8 values")
    p8 = dd.Plan(w.freqs, w.tsamp, w.nsamp, w.ranges, "u8")
    pf = dd.Plan(w.freqs, w.tsamp, w.nsamp, w.ranges, "f32")
    o8 = dd.dedisperse(torch.from_numpy(x).cuda(), p8)
    of = dd.dedisperse(torch.from_numpy(x.astype(np.float32)).cuda(), pf)
    torch.cuda.synchronize()
    assert torch.equal(o8.double(), of.double())


def test_adjoint_random_shapes_vs_oracle():
    for seed in range(4):
        x, freqs, tsamp, ranges, w = case(20 + seed)
        try:
            plan_o = O.expand_plan(freqs, tsamp, x.shape[1], ranges)
        except ValueError:
            continue
        say("f32 adjoint", seed, x.shape, ranges)
        plan = gpu_plan(freqs, tsamp, x.shape[1], ranges)
        rng = np.random.default_rng(40 + seed)
        g = rng.standard_normal(plan.out_elems).astype(np.float32)
        dx, dw = dd.adjoint(torch.from_numpy(g).cuda(), plan, x=torch.from_numpy(x).cuda(),
                            weights=torch.from_numpy(w).cuda())
        torch.cuda.synchronize()
        wX, ww = cref.adjoint_f32(x, freqs, tsamp, ranges, g.astype(np.float64), w)
        tX, tw = cref.adjoint_f32(np.abs(x), freqs, tsamp, ranges, np.abs(g).astype(np.float64),
                                  np.abs(w))
        check_close(dx.cpu().numpy().astype(np.float64), wX, tX, "dX")
        check_close(dw.cpu().numpy().astype(np.float64), ww, tw, "dw")
        assert len(plan_o) == len(ranges)


@pytest.mark.parametrize("nsamp,nch", [(5000, 70), (4001, 33), (1100, 1)])
def test_adjoint_one_range_full_resolution_vs_oracle(nsamp, nch):
    """Plans with one range at full resolution form dX and the weight
    gradient in the adjoint kernel's epilogue (no G buffer, no finalising
    pass): several time tiles with a ragged last one, output tiles of 32
    channels with a partial last one, and a one-channel plan."""
    x, freqs, tsamp, _, w = case(80 + nch, nch=nch, nsamp=nsamp)
    ranges = [(0.0, 45.0, 1.0, 1)]
    say("f32 fused adjoint", nsamp, nch)
    plan = gpu_plan(freqs, tsamp, nsamp, ranges)
    rng = np.random.default_rng(81)
    g = rng.standard_normal(plan.out_elems).astype(np.float32)
    xt, wt = torch.from_numpy(x).cuda(), torch.from_numpy(w).cuda()
    dx, dw = dd.adjoint(torch.from_numpy(g).cuda(), plan, x=xt, weights=wt)
    dx_only, none = dd.adjoint(torch.from_numpy(g).cuda(), plan, weights=wt, grad_w=False)
    torch.cuda.synchronize()
    assert none is None and torch.equal(dx, dx_only)
    wX, ww = cref.adjoint_f32(x, freqs, tsamp, ranges, g.astype(np.float64), w)
    tX, tw = cref.adjoint_f32(np.abs(x), freqs, tsamp, ranges, np.abs(g).astype(np.float64),
                              np.abs(w))
    check_close(dx.cpu().numpy().astype(np.float64), wX, tX, "dX")
    check_close(dw.cpu().numpy().astype(np.float64), ww, tw, "dw")


def test_adjoint_identity():
    """<A x, y> == <x, A^T y>: the GPU forward and the GPU adjoint are
    transposes (sums formed in FP64 on the host from the float32 results)."""
    x, freqs, tsamp, ranges, w = case(30, nch=64, nsamp=5000)
    say("adjoint identity")
    plan = gpu_plan(freqs, tsamp, x.shape[1], ranges)
    rng = np.random.default_rng(31)
    y = rng.standard_normal(plan.out_elems).astype(np.float32)
    xt, wt = torch.from_numpy(x).cuda(), torch.from_numpy(w).cuda()
    out = dd.dedisperse(xt, plan, weights=wt)
    dx, dw = dd.adjoint(torch.from_numpy(y).cuda(), plan, x=xt, weights=wt)
    torch.cuda.synchronize()
    lhs = float(np.dot(out.cpu().numpy().astype(np.float64), y.astype(np.float64)))
    rhs = float(np.sum(x.astype(np.float64) * dx.cpu().numpy()))
    rhs_w = float(np.dot(w.astype(np.float64), dw.cpu().numpy()))
    scale = float(np.sum(np.abs(y)) * np.abs(x).max() * np.abs(w).max() * x.shape[0])
    assert abs(lhs - rhs) <= 1e-6 * scale
    assert abs(lhs - rhs_w) <= 1e-6 * scale


def test_finite_differences():
    """The loss sum(g * out) is linear in w and x, so central differences of
    FP64-accumulated losses match the adjoint up to float32 rounding."""
    x, freqs, tsamp, ranges, w = case(40, nch=12, nsamp=1500)
    say("finite differences")
    plan = gpu_plan(freqs, tsamp, x.shape[1], ranges)
    rng = np.random.default_rng(41)
    g = rng.standard_normal(plan.out_elems).astype(np.float32)
    xt, wt, gt = torch.from_numpy(x).cuda(), torch.from_numpy(w).cuda(), torch.from_numpy(g).cuda()
    dx, dw = dd.adjoint(gt, plan, x=xt, weights=wt)

    def loss(xv, wv):
        o = dd.dedisperse(xv, plan, weights=wv)
        return float(np.dot(o.cpu().numpy().astype(np.float64), g.astype(np.float64)))

    h = 0.5
    for c in (0, 5, 11):
        e = torch.zeros_like(wt)
        e[c] = h
        fd = (loss(xt, wt + e) - loss(xt, wt - e)) / (2 * h)
        assert abs(fd - float(dw[c])) <= 1e-4 * max(1.0, abs(fd)), (c, fd, float(dw[c]))
    for (c, t) in ((0, 10), (6, 700), (11, 1499)):
        e = torch.zeros_like(xt)
        e[c, t] = h
        fd = (loss(xt + e, wt) - loss(xt - e, wt)) / (2 * h)
        assert abs(fd - float(dx[c, t])) <= 1e-4 * max(1.0, abs(fd)), (c, t, fd, float(dx[c, t]))


def test_autograd_function():
    x, freqs, tsamp, ranges, w = case(50, nch=40, nsamp=4000)
    say("autograd")
    plan = gpu_plan(freqs, tsamp, x.shape[1], ranges)
    rng = np.random.default_rng(51)
    g = torch.from_numpy(rng.standard_normal(plan.out_elems).astype(np.float32)).cuda()
    xt = torch.from_numpy(x).cuda().requires_grad_(True)
    wt = torch.from_numpy(w).cuda().requires_grad_(True)
    out = dd.dedisperse_autograd(xt, wt, plan)
    (out * g).sum().backward()
    dx, dw = dd.adjoint(g, plan, x=xt.detach(), weights=wt.detach())
    torch.cuda.synchronize()
    assert torch.equal(xt.grad, dx) and torch.equal(wt.grad, dw)
    wX, ww = cref.adjoint_f32(x, freqs, tsamp, ranges, g.cpu().numpy().astype(np.float64), w)
    assert normwise(xt.grad.cpu().numpy(), wX) <= RTOL
    assert normwise(wt.grad.cpu().numpy(), ww) <= RTOL


def test_differentiable_workload_full_size():
    """1024 channels x 2^16 float32, DM 0..511: forward and both gradients at
    full size against the FP64 C oracle."""
    w = synth.differentiable()
    say("differentiable workload: input")
    x = w.make_input()
    plan = gpu_plan(w.freqs, w.tsamp, w.nsamp, w.ranges)
    wts = np.ones(w.nchans, dtype=np.float32)
    g = synth.gaussian(w.seed, (plan.out_elems,))
    xt, wt, gt = (torch.from_numpy(x).cuda(), torch.from_numpy(wts).cuda(),
                  torch.from_numpy(g).cuda())
    say("differentiable workload: forward + adjoint")
    out = dd.dedisperse(xt, plan, weights=wt)
    dx, dw = dd.adjoint(gt, plan, x=xt, weights=wt)
    torch.cuda.synchronize()
    want = cref.dedisperse_f32(x, w.freqs, w.tsamp, w.ranges, wts)
    terms = cref.dedisperse_f32(np.abs(x), w.freqs, w.tsamp, w.ranges, wts)
    check_close(out.cpu().numpy().astype(np.float64), want, terms, "forward")
    wX, ww = cref.adjoint_f32(x, w.freqs, w.tsamp, w.ranges, g.astype(np.float64), wts)
    tX, tw = cref.adjoint_f32(np.abs(x), w.freqs, w.tsamp, w.ranges,
                              np.abs(g).astype(np.float64), wts)
    check_close(dx.cpu().numpy().astype(np.float64), wX, tX, "dX")
    check_close(dw.cpu().numpy().astype(np.float64), ww, tw, "dw")


def test_float_results_repeat_bit_identically():
    x, freqs, tsamp, ranges, w = case(60, nch=100, nsamp=5000)
    say("f32 determinism")
    plan = gpu_plan(freqs, tsamp, x.shape[1], ranges)
    xt, wt = torch.from_numpy(x).cuda(), torch.from_numpy(w).cuda()
    g = torch.randn(plan.out_elems, device="cuda", generator=torch.Generator("cuda").manual_seed(1))
    a = dd.dedisperse(xt, plan, weights=wt)
    b = dd.dedisperse(xt, plan, weights=wt)
    ga = dd.adjoint(g, plan, x=xt, weights=wt)
    gb = dd.adjoint(g, plan, x=xt, weights=wt)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    assert torch.equal(ga[0], gb[0]) and torch.equal(ga[1], gb[1])


@pytest.mark.parametrize("nsamp", [4000, 4001])
def test_unaligned_rows_vs_oracle(nsamp):
    """Input, gradient and dX rows that do not start on 16-byte boundaries
    (tensors at a one-float storage offset, and an odd series length) take
    the element-wise paths of the binning, padding and finalising kernels;
    their results must match the oracle as the aligned ones do."""
    x, freqs, tsamp, ranges, w = case(70, nch=24, nsamp=nsamp)
    say("f32 unaligned rows", nsamp)
    plan = gpu_plan(freqs, tsamp, nsamp, ranges)

    def shifted(a):
        flat = torch.zeros(a.size + 1, dtype=torch.float32, device="cuda")
        flat[1:] = torch.from_numpy(a.ravel()).cuda()
        return flat[1:].view(a.shape)

    xt, wt = shifted(x), torch.from_numpy(w).cuda()
    assert xt.data_ptr() % 16 != 0
    out = dd.dedisperse(xt, plan, weights=wt)
    rng = np.random.default_rng(71)
    g = rng.standard_normal(plan.out_elems).astype(np.float32)
    dx_buf = torch.zeros(x.size + 1, dtype=torch.float32, device="cuda")
    dx_view = dx_buf[1:].view(x.shape)
    dx, dw = dd.adjoint(shifted(g), plan, x=xt, weights=wt, grad_in=dx_view)
    torch.cuda.synchronize()
    want = cref.dedisperse_f32(x, freqs, tsamp, ranges, w)
    terms = cref.dedisperse_f32(np.abs(x), freqs, tsamp, ranges, np.abs(w))
    check_close(out.cpu().numpy().astype(np.float64), want, terms, "out")
    wX, ww = cref.adjoint_f32(x, freqs, tsamp, ranges, g.astype(np.float64), w)
    tX, tw = cref.adjoint_f32(np.abs(x), freqs, tsamp, ranges, np.abs(g).astype(np.float64),
                              np.abs(w))
    check_close(dx_view.cpu().numpy().astype(np.float64), wX, tX, "dX")
    check_close(dw.cpu().numpy().astype(np.float64), ww, tw, "dw")


def test_adjoint_rejects_integer_plans():
    w = synth.tiny()
    plan = dd.Plan(w.freqs, w.tsamp, w.nsamp, w.ranges, "u8")
    with pytest.raises(ValueError):
        dd.adjoint(torch.zeros(plan.out_elems, device="cuda"), plan)


def test_host_tensors_are_refused_before_any_launch():
    """Every tensor the binding hands to the library must live on the
    input's device: host tensors are refused with ValueError (a host address
    in a kernel would fault it)."""
    x, freqs, tsamp, ranges, w = case(1, nch=16, nsamp=2000)
    plan = gpu_plan(freqs, tsamp, x.shape[1], ranges)
    xd = torch.from_numpy(x).cuda()
    wd = torch.from_numpy(w).cuda()
    say("host tensors refused", plan.nchans, plan.nsamp)
    with pytest.raises(ValueError):
        dd.dedisperse(xd, plan, weights=torch.from_numpy(w))
    with pytest.raises(ValueError):
        dd.dedisperse(xd, plan, out=torch.empty(plan.out_elems, dtype=torch.float32))
    with pytest.raises(ValueError):
        dd.dedisperse(xd, plan, ws=torch.empty(plan.workspace_bytes, dtype=torch.uint8))
    g = torch.ones(plan.out_elems, device="cuda")
    with pytest.raises(ValueError):
        dd.adjoint(g, plan, x=torch.from_numpy(x), weights=wd)
    with pytest.raises(ValueError):
        dd.boxcar_loss(xd, plan, weights=wd, ws=torch.empty(plan.workspace_bytes, dtype=torch.uint8))
    s = dd.Stream(plan)
    with pytest.raises(ValueError):
        s.push(torch.zeros((plan.nchans, s.first), dtype=torch.uint8, device="cuda"))
    with pytest.raises(ValueError):
        s.push(torch.zeros((plan.nchans, s.first), dtype=torch.float32))
    # a workspace of another dtype counts in bytes
    ws = torch.empty((plan.workspace_bytes + 3) // 4, dtype=torch.float32, device="cuda")
    out = dd.dedisperse(xd, plan, weights=wd, ws=ws)
    ref = dd.dedisperse(xd, plan, weights=wd)
    torch.cuda.synchronize()
    assert torch.equal(out, ref)
