"""Integer variant 3 (exact sub-band reuse): bit-exact against the oracle
and identical to the direct kernel (variant 1) on the same input.

Plans whose delay patterns do not fit the LDS are rejected at plan
creation (DD_ERR_INVALID); those cases are skipped here and covered by the
host tests.  Every call goes through the C ABI on cuda:0.
"""
import numpy as np
import pytest

import synth
from oracle import cref
from oracle import dedisp as O

from test_forward_gpu import EDGES, oracle_flat, random_case, say

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
dd = pytest.importorskip("paper_1912_07704_amd")

CANARY = -123456789


def plan_v3(freqs, tsamp, nsamp, ranges, dm_tile=0, stage=0):
    try:
        return dd.Plan(freqs, tsamp, nsamp, ranges, "u8", variant=3, dm_tile=dm_tile,
                       stage_chans=stage)
    except dd.DDError as e:
        assert e.status == -2, e
        pytest.skip(f"delay patterns do not fit the LDS: {e}")


def forward(x, plan, extra=64):
    xt = torch.from_numpy(np.ascontiguousarray(x)).cuda()
    out = torch.full((plan.out_elems + extra,), CANARY, dtype=torch.int32, device="cuda")
    dd.dedisperse(xt, plan, out=out)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    assert (got[plan.out_elems:] == CANARY).all(), "wrote past out_elems"
    return got[: plan.out_elems]


@pytest.mark.parametrize("dm_tile", [128, 192, 96, 64])
@pytest.mark.parametrize("seed", range(16))
def test_random_shapes_bit_exact(seed, dm_tile):
    x, freqs, tsamp, ranges = random_case(seed)
    plan = plan_v3(freqs, tsamp, x.shape[1], ranges, dm_tile=dm_tile)
    say("variant 3 random", seed, dm_tile, x.shape, ranges, plan.strategy)
    got = forward(x, plan)
    assert np.array_equal(got, oracle_flat(x, freqs, tsamp, ranges))


@pytest.mark.parametrize("name", sorted(EDGES))
def test_edge_cases_bit_exact(name):
    nch, nsamp, ranges = EDGES[name]
    freqs = synth.band_freqs(1500.0, 1200.0, nch) if nch > 1 else np.array([1400.0])
    tsamp = 1e-3
    if name == "single_dm_single_sample":
        nsamp = int(O.shift_table(freqs, tsamp, [40.0]).max()) + 1
    if name == "wide_spread":
        freqs = synth.band_freqs(500.0, 300.0, nch)
    rng = np.random.default_rng(hash(name) % 2**32)
    x = rng.integers(0, 256, size=(nch, nsamp)).astype(np.uint8)
    if name == "downsample_256":
        x[:] = 255
    plan = plan_v3(freqs, tsamp, nsamp, ranges)
    say("variant 3 edge", name, x.shape, ranges, plan.strategy)
    got = forward(x, plan, extra=8)
    assert np.array_equal(got, oracle_flat(x, freqs, tsamp, ranges))


@pytest.mark.parametrize("stage", [16, 8])
def test_saturated_and_zero_input(stage):
    """Every sum at its bound (255*nchans*ds): the packed 16-bit halves of the
    partial-sum rows and of the accumulators never carry."""
    freqs = synth.band_freqs(1670.0, 1370.0, 1024)
    ranges = [(0.0, 40.0, 0.5, 1), (40.0, 80.0, 1.0, 16), (80.0, 100.0, 2.0, 32)]
    plan = plan_v3(freqs, 64e-6, 8192, ranges, stage=stage)
    for val in (255, 0):
        x = np.full((1024, 8192), val, dtype=np.uint8)
        say("variant 3 extreme", stage, val, plan.strategy)
        outs = plan.split(torch.from_numpy(forward(x, plan)))
        for ri, o in zip(plan.ranges, outs):
            assert (o == 255 * 1024 * ri.downsample * (val // 255)).all()


def test_small_workload_matches_direct_kernel():
    """A 300-channel band with fine DM steps (many shared patterns) at both
    DM tiles and stage widths: equal to variant 1 and to the oracle."""
    freqs = synth.band_freqs(1670.0, 1370.0, 300)
    ranges = [(0.0, 30.0, 0.1, 1), (30.0, 60.0, 0.2, 2)]
    rng = np.random.default_rng(11)
    x = rng.integers(0, 256, size=(300, 20000)).astype(np.uint8)
    want = cref.dedisperse_u8(x, freqs, 64e-6, ranges)
    p1 = dd.Plan(freqs, 64e-6, 20000, ranges, "u8", variant=1)
    assert np.array_equal(forward(x, p1), want)
    for dm_tile, stage in ((128, 0), (128, 8), (192, 0), (96, 0), (64, 0)):
        plan = plan_v3(freqs, 64e-6, 20000, ranges, dm_tile=dm_tile, stage=stage)
        say("variant 3 small workload", plan.strategy)
        assert np.array_equal(forward(x, plan), want)


def test_ska_full_size_equals_direct_kernel():
    """The SKA-like beam (4096 channels, 2^18 samples, 5 ranges): the whole
    output equals variant 1's, and sampled outputs equal the oracle's."""
    w = synth.ska_single_beam()
    say("variant 3 ska: input")
    x = w.make_input()
    xt = torch.from_numpy(x).cuda()
    p3 = plan_v3(w.freqs, w.tsamp, w.nsamp, w.ranges)
    p1 = dd.Plan(w.freqs, w.tsamp, w.nsamp, w.ranges, "u8", variant=1)
    say("variant 3 ska: forward", p3.strategy)
    o3 = dd.dedisperse(xt, p3)
    o1 = dd.dedisperse(xt, p1)
    torch.cuda.synchronize()
    assert torch.equal(o3, o1)
    op = O.expand_plan(w.freqs, w.tsamp, w.nsamp, w.ranges)
    rng = np.random.default_rng(78)
    outs = p3.split(o3)
    for r, ri in enumerate(p3.ranges):
        d = rng.integers(0, ri.ndms, 200)
        t = rng.integers(0, ri.nout, 200)
        t[:10] = ri.nout - 1 - np.arange(10)
        got = outs[r][torch.from_numpy(d).cuda(), torch.from_numpy(t).cuda()].cpu().numpy()
        assert np.array_equal(got, O.dedisperse_at(x, op, r, d, t))


def test_wide_channel_plan_equals_direct_kernel():
    """1024 wide channels at 128 us, DM 0..511 step 1, uint8: sub-band reuse
    fits at 128-DM tiles with one-sub-band stages (too many delay patterns
    for 192); the whole output equals variant 1's, and sampled outputs equal
    the oracle's."""
    w = synth.differentiable()
    rng = np.random.default_rng(512)
    x = rng.integers(0, 256, size=(1024, w.nsamp)).astype(np.uint8)
    xt = torch.from_numpy(x).cuda()
    p0 = plan_v3(w.freqs, w.tsamp, w.nsamp, w.ranges, dm_tile=128)
    assert p0.strategy["chans_stage"] == 8
    p1 = dd.Plan(w.freqs, w.tsamp, w.nsamp, w.ranges, "u8", variant=1)
    say("wide channels: variant 3", p0.strategy)
    o0 = dd.dedisperse(xt, p0)
    o1 = dd.dedisperse(xt, p1)
    torch.cuda.synchronize()
    assert torch.equal(o0, o1)
    op = O.expand_plan(w.freqs, w.tsamp, w.nsamp, w.ranges)
    ri = p0.ranges[0]
    d = rng.integers(0, ri.ndms, 300)
    t = rng.integers(0, ri.nout, 300)
    t[:10] = ri.nout - 1 - np.arange(10)
    out = p0.split(o0)[0]
    got = out[torch.from_numpy(d).cuda(), torch.from_numpy(t).cuda()].cpu().numpy()
    assert np.array_equal(got, O.dedisperse_at(x, op, 0, d, t))
