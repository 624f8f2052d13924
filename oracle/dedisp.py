"""Plain FP64 / int64 oracle for brute-force incoherent dedispersion.

TEST INFRASTRUCTURE ONLY: the product never imports this module.

The paper (Introduction) names dedispersion as the first analysis module of
the pipeline and cites its GPU implementation, but prints no formula.  The
operator written out here is the standard brute-force incoherent
dedispersion that the library implements:

* a DM plan is a list of ranges (lo, hi, step, downsample); range r holds
  the trial DMs lo + i*step for i < round((hi - lo)/step)  (half-open);
* every channel c is delayed by
  s[d][c] = floor(K * DM_d * (f_c^-2 - f_ref^-2) / (tsamp * ds) + 1/2)
  binned samples, with K = 4.148808e3 s MHz^2 pc^-1 cm^3 and f_ref the
  highest channel frequency;
* a range with downsample ds > 1 works on the series binned by summing ds
  adjacent samples (bin 0 = samples [0, ds), partial last bin dropped);
* out_r[d][t] = sum_c w_c * x_r[c][t + s[d][c]] for the valid samples
  t < nout_r = floor(nsamp / ds) - max_{d in r, c} s[d][c];
* ranges are concatenated in plan order, each DM-major [ndms_r][nout_r].

Integer input is summed in int64 (exact); float input in FP64.  The
adjoint and the boxcar loss follow the same definitions, transposed or
composed.  Nothing here is blocked, fused or reordered beyond the sums the
definition names.
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from fractions import Fraction

import numpy as np

K_DM = 4.148808e3   # s MHz^2 pc^-1 cm^3


# ---------------------------------------------------------------------------
# DM plan
# ---------------------------------------------------------------------------

@dataclass
class OracleRange:
    dms: np.ndarray      # float64 trial DMs of this range
    ds: int              # time downsampling factor
    shifts: np.ndarray   # int64 [ndms][nchans] delays in binned samples
    nbin: int            # floor(nsamp / ds)
    nout: int            # valid output samples per DM


def range_dms(lo: float, hi: float, step: float) -> np.ndarray:
    """Trial DMs of one half-open range: lo + i*step, i < round((hi-lo)/step).
    i*step is formed directly for every i (never accumulated)."""
    n = int(math.floor((hi - lo) / step + 0.5))
    return np.array([lo + i * step for i in range(n)], dtype=np.float64)


def shift_table(freqs, tsamp: float, dms, ds: int = 1) -> np.ndarray:
    """s[d][c] = floor(K*DM_d*(f_c^-2 - f_ref^-2)/(tsamp*ds) + 1/2), FP64,
    f_ref = max_c f_c.  Returned as int64 [ndms][nchans]."""
    freqs = np.asarray(freqs, dtype=np.float64)
    f_ref = float(freqs.max())
    delta = 1.0 / (freqs * freqs) - 1.0 / (f_ref * f_ref)
    dms = np.asarray(dms, dtype=np.float64)
    x = K_DM * dms[:, None] * delta[None, :] / (tsamp * ds)
    return np.floor(x + 0.5).astype(np.int64)


def shift_x_table(freqs, tsamp: float, dms, ds: int = 1) -> np.ndarray:
    """The unrounded delays x = K*DM*(f_c^-2 - f_ref^-2)/(tsamp*ds) in FP64
    (the quantity shift_table rounds)."""
    freqs = np.asarray(freqs, dtype=np.float64)
    f_ref = float(freqs.max())
    delta = 1.0 / (freqs * freqs) - 1.0 / (f_ref * f_ref)
    dms = np.asarray(dms, dtype=np.float64)
    return K_DM * dms[:, None] * delta[None, :] / (tsamp * ds)


def shift_exact(freq_c, freq_ref, tsamp, dm, ds: int = 1) -> int:
    """The same delay in exact rational arithmetic, starting from the FP64
    values of its inputs (each is converted to a Fraction without rounding).
    Used to pin the FP64 table where x lies close to a rounding tie."""
    K = Fraction(K_DM)
    fc = Fraction(float(freq_c))
    fr = Fraction(float(freq_ref))
    x = K * Fraction(float(dm)) * (1 / (fc * fc) - 1 / (fr * fr)) / (Fraction(float(tsamp)) * ds)
    return math.floor(x + Fraction(1, 2))


def shift_exact_x(freq_c, freq_ref, tsamp, dm, ds: int = 1) -> Fraction:
    K = Fraction(K_DM)
    fc = Fraction(float(freq_c))
    fr = Fraction(float(freq_ref))
    return K * Fraction(float(dm)) * (1 / (fc * fc) - 1 / (fr * fr)) / (Fraction(float(tsamp)) * ds)


def expand_plan(freqs, tsamp: float, nsamp: int, ranges) -> list:
    """Expand (lo, hi, step, ds) ranges into per-range DMs, shift tables and
    valid output lengths.  Raises ValueError when a range has no valid
    output sample."""
    out = []
    for (lo, hi, step, ds) in ranges:
        ds = int(ds)
        dms = range_dms(lo, hi, step)
        s = shift_table(freqs, tsamp, dms, ds)
        nbin = nsamp // ds
        smax = int(s.max()) if s.size else 0
        nout = nbin - smax
        if nout <= 0:
            raise ValueError("range has no valid output samples")
        out.append(OracleRange(dms, ds, s, nbin, nout))
    return out


def overlap_samples(plan) -> int:
    """Largest delay of the plan in native samples: the stride by which a
    streaming run must overlap consecutive chunks."""
    return max(int(r.shifts.max()) * r.ds for r in plan)


# ---------------------------------------------------------------------------
# Time downsampling
# ---------------------------------------------------------------------------

def decimate(x: np.ndarray, ds: int) -> np.ndarray:
    """x_ds[c][t'] = sum_{k<ds} x[c][ds*t' + k] for t' < floor(nsamp/ds).
    Integer input gives int64, float input gives float64."""
    x = np.asarray(x)
    acc_t = np.int64 if np.issubdtype(x.dtype, np.integer) else np.float64
    nch, nsamp = x.shape
    nbin = nsamp // ds
    out = np.zeros((nch, nbin), dtype=acc_t)
    for k in range(ds):
        out += x[:, k: k + ds * nbin: ds].astype(acc_t)
    return out


# ---------------------------------------------------------------------------
# Forward
# ---------------------------------------------------------------------------

def dedisperse_range(xr: np.ndarray, shifts: np.ndarray, nout: int,
                     weights=None) -> np.ndarray:
    """out[d][t] = sum_c w_c * xr[c][t + s[d][c]], t < nout, for an already
    binned input xr."""
    nd, nch = shifts.shape
    if np.issubdtype(xr.dtype, np.integer) and weights is None:
        acc_t = np.int64
    else:
        acc_t = np.float64
    out = np.zeros((nd, nout), dtype=acc_t)
    for d in range(nd):
        for c in range(nch):
            s = int(shifts[d, c])
            row = xr[c, s: s + nout].astype(acc_t)
            if weights is not None:
                row = row * float(weights[c])
            out[d] += row
    return out


def dedisperse(x: np.ndarray, freqs, tsamp: float, ranges, weights=None):
    """Full forward: returns (list of per-range outputs, plan)."""
    x = np.asarray(x)
    plan = expand_plan(freqs, tsamp, x.shape[1], ranges)
    outs = []
    for r in plan:
        xr = decimate(x, r.ds) if r.ds > 1 else x
        outs.append(dedisperse_range(xr, r.shifts, r.nout, weights))
    return outs, plan


def concat(outs) -> np.ndarray:
    """Ranges in plan order, each flattened DM-major."""
    return np.concatenate([o.ravel() for o in outs]) if outs else np.zeros(0)


def dedisperse_at(x: np.ndarray, plan, r: int, d_idx, t_idx, weights=None):
    """Selected outputs out_r[d][t] computed one by one straight from the
    native-resolution input (the bin sums are formed per output), for
    full-size checks where the complete output is too large."""
    x = np.asarray(x)
    rr = plan[r]
    ds = rr.ds
    nch = x.shape[0]
    integer = np.issubdtype(x.dtype, np.integer) and weights is None
    res = np.zeros(len(d_idx), dtype=np.int64 if integer else np.float64)
    chans = np.arange(nch)
    for i, (d, t) in enumerate(zip(d_idx, t_idx)):
        base = (int(t) + rr.shifts[int(d)]) * ds          # native start per channel
        tot = np.zeros(nch, dtype=np.int64 if integer else np.float64)
        for k in range(ds):
            tot += x[chans, base + k].astype(tot.dtype)
        if weights is not None:
            tot = tot * np.asarray(weights, dtype=np.float64)
        res[i] = tot.sum()
    return res


# ---------------------------------------------------------------------------
# Adjoint (transpose of the forward map, per range then summed)
# ---------------------------------------------------------------------------

def adjoint(g_outs, x: np.ndarray, plan, weights, nsamp: int):
    """Gradients of L = sum_r <g_r, out_r> with respect to x and w.

    G_r[c][tau] = sum_{d in r, 0 <= tau - s[d][c] < nout_r} g_r[d][tau - s[d][c]]
    dX[c][ds*tau + k] += w_c * G_r[c][tau]  (k < ds; samples past the last
    full bin get nothing)
    dw_c = sum_r sum_tau x_r[c][tau] * G_r[c][tau]
    """
    nch = len(weights)
    w = np.asarray(weights, dtype=np.float64)
    dX = np.zeros((nch, nsamp), dtype=np.float64)
    dw = np.zeros(nch, dtype=np.float64)
    for rr, g in zip(plan, g_outs):
        g = np.asarray(g, dtype=np.float64)
        G = np.zeros((nch, rr.nbin), dtype=np.float64)
        for d in range(len(rr.dms)):
            for c in range(nch):
                s = int(rr.shifts[d, c])
                G[c, s: s + rr.nout] += g[d]
        xr = decimate(x, rr.ds) if rr.ds > 1 else np.asarray(x, dtype=np.float64)
        dw += (xr * G).sum(axis=1)
        for k in range(rr.ds):
            dX[:, k: k + rr.ds * rr.nbin: rr.ds] += w[:, None] * G
    return dX, dw


# ---------------------------------------------------------------------------
# Boxcar loss on the dedispersed series
# ---------------------------------------------------------------------------

BOXCAR_WIDTHS = (1, 2, 4, 8, 16, 32)


def boxcar_sums(row: np.ndarray, w: int) -> np.ndarray:
    """B[t] = sum_{k<w} row[t+k] for the valid windows t <= len(row) - w."""
    n = len(row) - w + 1
    if n <= 0:
        return np.zeros(0, dtype=np.float64)
    B = np.zeros(n, dtype=np.float64)
    for k in range(w):
        B += row[k: k + n]
    return B


def boxcar_loss(outs, widths=BOXCAR_WIDTHS) -> float:
    """L = sum_r sum_d sum_w sum_t (boxcar_w(out_r[d])[t])^2."""
    L = 0.0
    for o in outs:
        o = np.asarray(o, dtype=np.float64)
        for d in range(o.shape[0]):
            for w in widths:
                B = boxcar_sums(o[d], w)
                L += float((B * B).sum())
    return L


def boxcar_loss_grad(outs, widths=BOXCAR_WIDTHS):
    """dL/dout: each window t of width w sends 2*B_w[t] to the samples it
    covers."""
    grads = []
    for o in outs:
        o = np.asarray(o, dtype=np.float64)
        g = np.zeros_like(o)
        for d in range(o.shape[0]):
            for w in widths:
                B = boxcar_sums(o[d], w)
                for k in range(w):
                    g[d, k: k + len(B)] += 2.0 * B
        grads.append(g)
    return grads
