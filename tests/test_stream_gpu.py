"""Streaming in chunks with the plan's largest delay as overlap (the
pipeline's chunked iterations, paper "Pipeline"), and the corner turn from
time-major blocks: the concatenated chunks equal the CPU oracle over the
whole series (bit for bit for uint8, within the float32 tolerance for
float32) and reproduce one forward over the whole series."""
import numpy as np
import pytest

import synth
from oracle import cref

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
dd = pytest.importorskip("paper_1912_07704_amd")


def say(*a):
    print("[case]", *a, flush=True)


def series_case(dtype, nchunks=4, seed=0):
    freqs = synth.band_freqs(1670.0, 1370.0, 256)
    tsamp = 256e-6
    ranges = [(0.0, 100.0, 1.0, 1), (100.0, 300.0, 2.0, 2), (300.0, 400.0, 5.0, 4)]
    nsamp = 16384
    plan = dd.Plan(freqs, tsamp, nsamp, ranges, dtype)
    s = dd.Stream(plan)
    total = nsamp + (nchunks - 1) * s.step
    rng = np.random.default_rng(seed)
    if dtype == "u8":
        x = rng.integers(0, 256, size=(256, total)).astype(np.uint8)
    else:
        x = rng.standard_normal((256, total)).astype(np.float32)
    return freqs, tsamp, ranges, plan, s, x


@pytest.mark.parametrize("dtype,time_major", [("u8", False), ("u8", True), ("f32", False),
                                              ("f32", True)])
def test_stream_equals_one_shot(dtype, time_major):
    freqs, tsamp, ranges, plan, s, x = series_case(dtype)
    if time_major:
        s = dd.Stream(plan, time_major=True)
    say("stream", dtype, "time-major" if time_major else "channel-major", x.shape, s.step)
    xt = torch.from_numpy(x).cuda()
    full = dd.Plan(freqs, tsamp, x.shape[1], ranges, dtype)
    want = [o.clone() for o in full.split(dd.dedisperse(xt, full))]
    got = [[] for _ in ranges]
    k = 0
    while plan.nsamp + k * s.step <= x.shape[1]:
        # chunk k covers [k*step, k*step + nsamp); its new samples are the
        # whole chunk for k = 0, then the last `step` samples
        lo = 0 if k == 0 else plan.nsamp + (k - 1) * s.step
        hi = plan.nsamp + k * s.step
        blk = xt[:, lo:hi]
        blk = blk.t().contiguous() if time_major else blk.contiguous()
        idx, out = s.push(blk)
        assert idx == k
        for r, e in enumerate(s.emitted(out)):
            got[r].append(e.clone())
        k += 1
    torch.cuda.synchronize()
    assert k == 4
    # the oracle over the whole series, split per range
    if dtype == "u8":
        ref = cref.dedisperse_u8(x, freqs, tsamp, ranges)
    else:
        ref = cref.dedisperse_f32(x, freqs, tsamp, ranges)
        terms = cref.dedisperse_f32(np.abs(x), freqs, tsamp, ranges)
    for r in range(len(ranges)):
        g = torch.cat(got[r], dim=1)
        assert g.shape[1] == 4 * (s.step // plan.ranges[r].downsample)
        assert torch.equal(g, want[r][:, : g.shape[1]]), f"range {r}"
        gn = g.cpu().numpy()
        wr = full.split(ref)[r][:, : gn.shape[1]]
        if dtype == "u8":
            assert np.array_equal(gn, wr), f"range {r} vs oracle"
        else:
            tr = full.split(terms)[r][:, : gn.shape[1]]
            err = np.abs(gn.astype(np.float64) - wr)
            nw = float(err.max() / np.abs(wr).max())
            assert nw <= 1e-5, f"range {r}: normwise {nw:.3e}"
            assert not (err > 1e-5 * tr + 1e-30).any(), f"range {r}: elementwise bound"


def test_stream_rejects_wrong_block_sizes():
    _, _, _, plan, s, x = series_case("u8", nchunks=2)
    xt = torch.from_numpy(x).cuda()
    with pytest.raises(dd.DDError):
        s.push(xt[:, : s.step].contiguous())            # the first push needs nsamp samples
    s.push(xt[:, : plan.nsamp].contiguous())
    with pytest.raises(dd.DDError):
        s.push(xt[:, : plan.nsamp].contiguous())        # later pushes need step samples
    s.reset()
    s.push(xt[:, : plan.nsamp].contiguous())


@pytest.mark.parametrize("shape", [(1, 1), (31, 33), (1000, 257), (4096, 64), (77, 4096)])
def test_corner_turn(shape):
    rng = np.random.default_rng(sum(shape))
    for dt in (np.uint8, np.float32):
        x = (rng.integers(0, 256, size=shape) if dt == np.uint8 else rng.standard_normal(shape))
        x = x.astype(dt)
        say("corner turn", shape, dt.__name__)
        got = dd.corner_turn(torch.from_numpy(x).cuda())
        torch.cuda.synchronize()
        assert np.array_equal(got.cpu().numpy(), x.T)
