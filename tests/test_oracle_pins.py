"""Pins of the CPU oracle against facts that do not come from the oracle.

Each test names what would fail if the oracle had a plausible mistake:
a dropped reference-frequency term, a wrong sign, a transposed index, a
mean instead of a sum in the binning, an off-by-one output length, and so on.
"""
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import synth
from oracle import cref
from oracle import dedisp as O

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def small_case(seed, nch=6, nsamp=96, ranges=((0.0, 6.0, 1.5, 1), (6.0, 12.0, 2.0, 3))):
    rng = np.random.default_rng(seed)
    freqs = np.sort(rng.uniform(1000.0, 1500.0, nch))[::-1].copy()
    x = rng.integers(0, 256, size=(nch, nsamp)).astype(np.uint8)
    return x, freqs, 1e-3, list(ranges)


# ---------------------------------------------------------------------------
# Shift table: closed forms, exact rationals, physical units
# ---------------------------------------------------------------------------

def test_shift_units_and_constant_closed_forms():
    # DM 1 at 1000 MHz against a reference so high its term is 1e-12 of the
    # other: x = 4148.808 * (1e-6 - 1e-12) / 1e-6 = 4148.8038..., rounds to 4149.
    s = O.shift_table([1.0e6, 1000.0], 1e-6, [1.0])
    assert s.tolist() == [[0, 4149]]
    # 1/1200^2 - 1/1500^2 = 810000/(1440000*2250000) = 2.5e-7 exactly, so at
    # DM 100 and 128 us: x = 414880.8 * 2.5e-7 / 1.28e-4 = 810.3140625 -> 810;
    # with 4x binning x = 202.578515625 -> 203.
    assert O.shift_table([1500.0, 1200.0], 128e-6, [100.0]).tolist() == [[0, 810]]
    assert O.shift_table([1500.0, 1200.0], 128e-6, [100.0], ds=4).tolist() == [[0, 203]]
    # Order of channels does not matter: the reference is the maximum.
    assert O.shift_table([1200.0, 1500.0], 128e-6, [100.0]).tolist() == [[810, 0]]


def test_shift_zero_cases_and_monotone():
    w = synth.tiny()
    dms = O.range_dms(0.0, 100.0, 1.0)
    s = O.shift_table(w.freqs, w.tsamp, dms)
    assert (s[0] == 0).all()                       # DM 0
    assert (s[:, int(np.argmax(w.freqs))] == 0).all()   # reference channel
    assert (s >= 0).all()
    assert (np.diff(s, axis=0) >= 0).all()         # non-decreasing in DM
    assert (np.diff(s, axis=1) >= 0).all()         # descending band -> growing delay


def test_shift_table_equals_exact_rationals_small_plan():
    x, freqs, tsamp, ranges = small_case(1, nch=7)
    for (lo, hi, step, ds) in ranges:
        dms = O.range_dms(lo, hi, step)
        s = O.shift_table(freqs, tsamp, dms, ds)
        f_ref = freqs.max()
        for d, dm in enumerate(dms):
            for c, f in enumerate(freqs):
                assert s[d, c] == O.shift_exact(f, f_ref, tsamp, dm, ds)


def test_shift_near_ties_golden():
    rows = [ln.split() for ln in open(os.path.join(GOLDEN, "shift_near_ties.txt"))
            if not ln.startswith("#")]
    assert len(rows) > 20
    wls = {w.name: w for w in [synth.tiny(), synth.ska_single_beam(), synth.differentiable(),
                               synth.batched_differentiable(1)[0]]}
    for name, r, d, c, dm, f, s_exact, _ in rows:
        w = wls[name]
        lo, hi, step, ds = w.ranges[int(r)]
        dms = O.range_dms(lo, hi, step)
        assert dms[int(d)] == float(dm)
        assert w.freqs[int(c)] == float(f)
        s = O.shift_table(w.freqs, w.tsamp, dms[int(d): int(d) + 1], ds)[0, int(c)]
        assert s == int(s_exact)


def test_dm_grid_half_open():
    assert len(O.range_dms(0.0, 100.0, 1.0)) == 100
    assert len(O.range_dms(0.0, 150.0, 0.1)) == 1500
    d = O.range_dms(150.0, 300.0, 0.2)
    assert len(d) == 750 and d[0] == 150.0 and abs(d[-1] - 299.8) < 1e-9
    # i*step is formed directly, not accumulated
    assert d[500] == 150.0 + 500 * 0.2


def test_reference_plan_sizes():
    """Per-range DM counts, largest delays and valid lengths of the tiny and
    SKA-like plans; the largest delay is checked against exact rationals at
    the extreme (highest DM, lowest channel) entry."""
    w = synth.tiny()
    plan = O.expand_plan(w.freqs, w.tsamp, w.nsamp, w.ranges)
    assert [(len(r.dms), int(r.shifts.max()), r.nout) for r in plan] == [(100, 397, 65139)]
    w = synth.ska_single_beam()
    plan = O.expand_plan(w.freqs, w.tsamp, w.nsamp, w.ranges)
    got = [(len(r.dms), int(r.shifts.max()), r.nout) for r in plan]
    assert got == [(1500, 1692, 260452), (750, 1692, 129380), (400, 1410, 64126),
                   (500, 1410, 31358), (500, 1410, 14974)]
    f_ref = w.freqs.max()
    for r, (lo, hi, step, ds) in zip(plan, w.ranges):
        assert int(r.shifts.max()) == O.shift_exact(w.freqs.min(), f_ref, w.tsamp, r.dms[-1], ds)
    assert sum(len(r.dms) * r.nout for r in plan) == 536529400
    assert O.overlap_samples(plan) == 22560


# ---------------------------------------------------------------------------
# The sum: brute force, impulse response, invariants
# ---------------------------------------------------------------------------

def explicit_matrix(nch, nsamp, plan):
    """The operator as a 0/1 matrix built entry by entry from its impulse
    response: input sample (c, tau) reaches output (d, t) of range r iff
    tau // ds == t + s[d][c] and tau lies in a complete bin."""
    rows = sum(len(r.dms) * r.nout for r in plan)
    A = np.zeros((rows, nch * nsamp), dtype=np.int64)
    row0 = 0
    for r in plan:
        for d in range(len(r.dms)):
            for t in range(r.nout):
                for c in range(nch):
                    for tau in range(r.ds * r.nbin):
                        if tau // r.ds == t + r.shifts[d, c]:
                            A[row0 + d * r.nout + t, c * nsamp + tau] = 1
        row0 += len(r.dms) * r.nout
    return A


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_brute_force_matrix(seed):
    x, freqs, tsamp, ranges = small_case(seed, nch=4, nsamp=40,
                                         ranges=((0.0, 4.0, 1.0, 1), (4.0, 8.0, 2.0, 3)))
    outs, plan = O.dedisperse(x, freqs, tsamp, ranges)
    A = explicit_matrix(x.shape[0], x.shape[1], plan)
    assert np.array_equal(O.concat(outs), A @ x.ravel().astype(np.int64))


def test_impulse_response():
    nch, nsamp = 5, 80
    _, freqs, tsamp, ranges = small_case(3, nch=nch, nsamp=nsamp)
    plan = O.expand_plan(freqs, tsamp, nsamp, ranges)
    for (c, tau) in [(0, 7), (4, 33), (2, 60), (3, 79)]:
        x = np.zeros((nch, nsamp), dtype=np.uint8)
        x[c, tau] = 1
        outs, _ = O.dedisperse(x, freqs, tsamp, ranges)
        for r, o in zip(plan, outs):
            want = np.zeros_like(o)
            for d in range(len(r.dms)):
                t = tau // r.ds - r.shifts[d, c]
                if tau < r.ds * r.nbin and 0 <= t < r.nout:
                    want[d, t] = 1
            assert np.array_equal(o, want)


def test_dm_zero_row_is_channel_sum():
    w = synth.tiny()
    x = w.make_input()[:, :4096]
    outs, plan = O.dedisperse(x, w.freqs, w.tsamp, [(0.0, 3.0, 1.0, 1)])
    nout = plan[0].nout
    assert np.array_equal(outs[0][0], x[:, :nout].astype(np.int64).sum(axis=0))


def test_constant_input():
    x, freqs, tsamp, ranges = small_case(4)
    x[:] = 7
    outs, _ = O.dedisperse(x, freqs, tsamp, ranges)
    for o, (_, _, _, ds) in zip(outs, ranges):
        assert (o == x.shape[0] * ds * 7).all()


def test_decimation_is_a_sum_of_adjacent_samples():
    rng = np.random.default_rng(5)
    x = rng.integers(0, 256, size=(3, 103)).astype(np.uint8)
    for ds in (1, 2, 3, 16):
        nbin = 103 // ds
        want = np.add.reduceat(x[:, :nbin * ds].astype(np.int64), np.arange(0, nbin * ds, ds), axis=1)
        assert np.array_equal(O.decimate(x, ds), want)


def test_binned_range_equals_native_oracle_on_binned_input():
    x, freqs, tsamp, _ = small_case(6, nch=5, nsamp=120)
    ds = 4
    outs, _ = O.dedisperse(x, freqs, tsamp, [(0.0, 10.0, 2.5, ds)])
    xb = O.decimate(x, ds)
    ref, _ = O.dedisperse(xb, freqs, tsamp * ds, [(0.0, 10.0, 2.5, 1)])
    assert np.array_equal(outs[0], ref[0])


def test_linearity_exact():
    x, freqs, tsamp, ranges = small_case(7)
    rng = np.random.default_rng(8)
    y = rng.integers(0, 256, size=x.shape).astype(np.int64)
    a, b = 3, -5
    ox, _ = O.dedisperse(x.astype(np.int64), freqs, tsamp, ranges)
    oy, _ = O.dedisperse(y, freqs, tsamp, ranges)
    oz, _ = O.dedisperse(a * x.astype(np.int64) + b * y, freqs, tsamp, ranges)
    for p, q, z in zip(ox, oy, oz):
        assert np.array_equal(z, a * p + b * q)


def test_channel_permutation_invariance():
    x, freqs, tsamp, ranges = small_case(9, nch=8)
    perm = np.random.default_rng(10).permutation(8)
    o1, _ = O.dedisperse(x, freqs, tsamp, ranges)
    o2, _ = O.dedisperse(x[perm], freqs[perm], tsamp, ranges)
    for p, q in zip(o1, o2):
        assert np.array_equal(p, q)


def test_time_shift_equivariance():
    x, freqs, tsamp, ranges = small_case(11, nch=5, nsamp=150)
    m = 2     # bins; the input moves by m * ds native samples per range
    for rg in ranges:
        ds = rg[3]
        o1, p1 = O.dedisperse(x, freqs, tsamp, [rg])
        o2, p2 = O.dedisperse(x[:, m * ds:], freqs, tsamp, [rg])
        n = p2[0].nout
        assert np.array_equal(o1[0][:, m: m + n], o2[0])


def test_pulse_closed_form_tiny():
    """A pulse on the DM grid, unclipped, sums to nchans*amp on its own DM
    row for each of its samples: 128 * 48 = 6144."""
    w = synth.tiny()
    p = w.pulses[0]
    img = synth.pulse_image(w.freqs, w.tsamp, w.nsamp, w.pulses)
    outs, _ = O.dedisperse(img, w.freqs, w.tsamp, w.ranges)
    row = outs[0][50]
    assert (row[p.t0: p.t0 + p.width] == 128 * 48).all()
    assert row.max() == 6144 and (row == 6144).sum() == 4
    # noise + pulse minus noise is the pulse-only output (no clipping here)
    noisy = w.make_input()
    clean = synth.noise_only_u8(w.seed, w.freqs, w.tsamp, w.nsamp)
    assert np.array_equal(noisy.astype(np.int32) - clean, img)


def test_pulse_recovery_tiny():
    w = synth.tiny()
    p = w.pulses[0]
    outs, plan = O.dedisperse(w.make_input(), w.freqs, w.tsamp, w.ranges)
    o = outs[0].astype(np.float64)
    o -= o.mean(axis=1, keepdims=True)
    box = o[:, :-3] + o[:, 1:-2] + o[:, 2:-1] + o[:, 3:]
    d, t = np.unravel_index(np.argmax(box), box.shape)
    assert abs(plan[0].dms[d] - p.dm) <= 1.0 and abs(t - p.t0) <= p.width


def test_pulse_recovery_ska_first_pulses():
    """Recovery of the injected SKA-like pulses at their DM and arrival time
    on a reduced channel count (512 channels keep the oracle fast); the DM
    tolerance is the trial step plus the pulse-width smear in DM."""
    w = synth.ska_single_beam(nchans=512)
    x = w.make_input()
    plan = O.expand_plan(w.freqs, w.tsamp, w.nsamp, w.ranges)
    f = w.freqs
    dmax = 1.0 / f.min() ** 2 - 1.0 / f.max() ** 2
    for p in w.pulses[:2]:
        r = next(i for i, rg in enumerate(w.ranges) if rg[0] <= p.dm < rg[1])
        rr = plan[r]
        ds = rr.ds
        # only the DMs near the pulse (keeps the oracle cheap)
        di = np.nonzero(np.abs(rr.dms - p.dm) < 25.0)[0]
        xr = O.decimate(x, ds) if ds > 1 else x
        out = O.dedisperse_range(xr, rr.shifts[di], rr.nout).astype(np.float64)
        out -= out.mean(axis=1, keepdims=True)
        wb = max(1, math.ceil(p.width / ds))
        cs = np.cumsum(np.pad(out, ((0, 0), (1, 0))), axis=1)
        box = cs[:, wb:] - cs[:, :-wb]
        lo_t = max(0, p.t0 // ds - 200)
        hi_t = min(box.shape[1], p.t0 // ds + 200)
        sub = box[:, lo_t:hi_t]
        d, t = np.unravel_index(np.argmax(sub), sub.shape)
        dm_found = rr.dms[di[d]]
        tol = (w.ranges[r][2] + p.width * w.tsamp / (O.K_DM * dmax)) * 1.5
        assert abs(dm_found - p.dm) <= tol, (p, dm_found)
        assert abs((t + lo_t) * ds - p.t0) <= p.width + ds, (p, t + lo_t)


# ---------------------------------------------------------------------------
# Two oracles agree (numpy vs plain C)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("seed", range(4))
def test_c_oracle_matches_numpy_oracle_small(seed):
    rng = np.random.default_rng(100 + seed)
    nch = int(rng.integers(1, 40))
    nsamp = int(rng.integers(200, 3000))
    freqs = np.sort(rng.uniform(300.0, 1600.0, nch))[::-1].copy()
    ranges = [(0.0, 20.0, 0.5, 1), (20.0, 40.0, 1.0, 2), (40.0, 50.0, 2.0, 5)]
    x = rng.integers(0, 256, size=(nch, nsamp)).astype(np.uint8)
    try:
        outs, _ = O.dedisperse(x, freqs, 1e-3, ranges)
    except ValueError:
        with pytest.raises(ValueError):
            cref.dedisperse_u8(x, freqs, 1e-3, ranges)
        return
    assert np.array_equal(cref.dedisperse_u8(x, freqs, 1e-3, ranges), O.concat(outs))
    xf = rng.standard_normal((nch, nsamp)).astype(np.float32)
    wts = rng.uniform(0.5, 1.5, nch).astype(np.float32)
    of, _ = O.dedisperse(xf, freqs, 1e-3, ranges, weights=wts.astype(np.float64))
    np.testing.assert_allclose(cref.dedisperse_f32(xf, freqs, 1e-3, ranges, wts),
                               O.concat(of), rtol=1e-12, atol=1e-9)
    for (lo, hi, st, ds) in ranges:
        assert np.array_equal(cref.range_shifts(freqs, 1e-3, (lo, hi, st, ds)),
                              O.shift_table(freqs, 1e-3, O.range_dms(lo, hi, st), ds))


def test_c_oracle_matches_numpy_oracle_tiny_workload():
    w = synth.tiny()
    x = w.make_input()
    outs, _ = O.dedisperse(x, w.freqs, w.tsamp, w.ranges)
    assert np.array_equal(cref.dedisperse_u8(x, w.freqs, w.tsamp, w.ranges), O.concat(outs))


def test_sampled_outputs_match_full_oracle():
    x, freqs, tsamp, ranges = small_case(12, nch=9, nsamp=300)
    outs, plan = O.dedisperse(x, freqs, tsamp, ranges)
    rng = np.random.default_rng(13)
    for r, o in enumerate(outs):
        d = rng.integers(0, o.shape[0], 30)
        t = rng.integers(0, o.shape[1], 30)
        assert np.array_equal(O.dedisperse_at(x, plan, r, d, t), o[d, t])


# ---------------------------------------------------------------------------
# Adjoint and boxcar loss
# ---------------------------------------------------------------------------

def test_adjoint_identity_exact_integers():
    """<A x, y> == <x, A^T y> for integer x, y (exact in int64 / FP64 here)."""
    x, freqs, tsamp, ranges = small_case(14, nch=6, nsamp=130)
    rng = np.random.default_rng(15)
    outs, plan = O.dedisperse(x.astype(np.int64), freqs, tsamp, ranges)
    ys = [rng.integers(-50, 50, size=o.shape) for o in outs]
    lhs = sum(int((o * y).sum()) for o, y in zip(outs, ys))
    w = np.ones(x.shape[0])
    dX, dw = O.adjoint(ys, x, plan, w, x.shape[1])
    assert dX.dtype == np.float64
    assert lhs == int((x.astype(np.int64) * dX.astype(np.int64)).sum())
    # with unit weights the weight gradient equals <A x, y> split by channel
    assert abs(dw.sum() - lhs) < 1e-6


def test_adjoint_matches_explicit_transpose():
    x, freqs, tsamp, ranges = small_case(16, nch=4, nsamp=40,
                                         ranges=((0.0, 4.0, 1.0, 1), (4.0, 8.0, 2.0, 3)))
    plan = O.expand_plan(freqs, tsamp, x.shape[1], ranges)
    A = explicit_matrix(x.shape[0], x.shape[1], plan)
    rng = np.random.default_rng(17)
    y = rng.standard_normal(A.shape[0])
    ys, off = [], 0
    for r in plan:
        n = len(r.dms) * r.nout
        ys.append(y[off: off + n].reshape(len(r.dms), r.nout))
        off += n
    w = rng.uniform(0.5, 2.0, x.shape[0])
    dX, dw = O.adjoint(ys, x, plan, w, x.shape[1])
    np.testing.assert_allclose(dX.ravel(), (A.T @ y) * np.repeat(w, x.shape[1]), rtol=1e-12)


@pytest.mark.parametrize("seed", range(3))
def test_c_adjoint_matches_numpy_adjoint(seed):
    rng = np.random.default_rng(300 + seed)
    nch = int(rng.integers(1, 20))
    nsamp = int(rng.integers(300, 1500))
    freqs = np.sort(rng.uniform(1000.0, 1500.0, nch))[::-1].copy()
    ranges = [(0.0, 8.0, 1.0, 1), (8.0, 16.0, 2.0, 3)]
    x = rng.standard_normal((nch, nsamp)).astype(np.float32)
    w = rng.uniform(0.5, 1.5, nch).astype(np.float32)
    plan = O.expand_plan(freqs, 1e-3, nsamp, ranges)
    gs = [rng.standard_normal((len(r.dms), r.nout)) for r in plan]
    dX, dw = O.adjoint(gs, x.astype(np.float64), plan, w.astype(np.float64), nsamp)
    cX, cw = cref.adjoint_f32(x, freqs, 1e-3, ranges, O.concat(gs), w)
    np.testing.assert_allclose(cX, dX, rtol=1e-12, atol=1e-10)
    np.testing.assert_allclose(cw, dw, rtol=1e-12, atol=1e-9)


def test_weight_gradient_finite_differences():
    """L(w) = sum g * out(w) is linear in w, so central differences are exact
    up to rounding."""
    rng = np.random.default_rng(18)
    _, freqs, tsamp, ranges = small_case(19, nch=5, nsamp=90)
    x = rng.standard_normal((5, 90))
    w = rng.uniform(0.5, 1.5, 5)
    outs, plan = O.dedisperse(x, freqs, tsamp, ranges, weights=w)
    gs = [rng.standard_normal(o.shape) for o in outs]
    dX, dw = O.adjoint(gs, x, plan, w, 90)

    def loss(wv, xv):
        o, _ = O.dedisperse(xv, freqs, tsamp, ranges, weights=wv)
        return sum(float((a * b).sum()) for a, b in zip(o, gs))

    h = 1e-3
    for c in range(5):
        e = np.zeros(5)
        e[c] = h
        fd = (loss(w + e, x) - loss(w - e, x)) / (2 * h)
        assert abs(fd - dw[c]) < 1e-8 * max(1.0, abs(fd))
    for (c, t) in [(0, 3), (2, 50), (4, 89)]:
        e = np.zeros_like(x)
        e[c, t] = h
        fd = (loss(w, x + e) - loss(w, x - e)) / (2 * h)
        assert abs(fd - dX[c, t]) < 1e-8 * max(1.0, abs(fd))


def test_boxcar_prefix_sum_and_fd():
    rng = np.random.default_rng(20)
    outs = [rng.standard_normal((3, 70)), rng.standard_normal((2, 40))]
    for o in outs:
        cs = np.concatenate([[0.0], np.cumsum(o[0])])
        for w in (1, 2, 4, 8, 16, 32):
            np.testing.assert_allclose(O.boxcar_sums(o[0], w), cs[w:] - cs[:-w], atol=1e-12)
    L = O.boxcar_loss(outs)
    g = O.boxcar_loss_grad(outs)
    h = 1e-4
    for (r, d, t) in [(0, 0, 0), (0, 2, 35), (1, 1, 39), (1, 0, 20)]:
        op = [o.copy() for o in outs]
        om = [o.copy() for o in outs]
        op[r][d, t] += h
        om[r][d, t] -= h
        fd = (O.boxcar_loss(op) - O.boxcar_loss(om)) / (2 * h)
        assert abs(fd - g[r][d, t]) < 1e-6 * max(1.0, abs(fd))
    # width 1 alone is the sum of squares
    assert abs(O.boxcar_loss(outs, (1,)) - sum(float((o * o).sum()) for o in outs)) < 1e-9
