"""Seeded synthetic filterbanks and workload descriptions.

This module is shared by the tests, the benchmark and the smoke check.  It
simulates *input data* only: Gaussian radiometer noise, the channel frequency
grid, and dispersed pulses placed with the cold-plasma delay law (the sky
signal that dedispersion later undoes).  It contains no dedispersion: no DM
plan expansion, no shift table, no decimation and no shift-and-sum.

Every array is a pure function of a seed.  Substreams come from
``numpy.random.SeedSequence(seed).spawn``; the noise of each 64-channel block
has its own substream, so the bytes do not depend on how many threads made
them.
"""
from __future__ import annotations

import math
import os
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass, field

import numpy as np

# Cold-plasma dispersion constant in s MHz^2 pc^-1 cm^3 (the value the
# dedispersion problem statement fixes).
K_DISP = 4.148808e3

NOISE_BLOCK = 64          # channels per noise substream
_STREAMS = ("noise", "pulses", "grad", "beams", "weights")


def _substreams(seed: int) -> dict:
    kids = np.random.SeedSequence(seed).spawn(len(_STREAMS))
    return dict(zip(_STREAMS, kids))


def _threads() -> int:
    return max(1, min(16, os.cpu_count() or 1))


# --------------------------------------------------------------------------
# Frequencies and the sky model
# --------------------------------------------------------------------------

def channel_freqs(f_hi: float, foff: float, nchans: int) -> np.ndarray:
    """SIGPROC-style channel grid: f_c = f_hi + c * foff (foff < 0 for a
    descending band)."""
    return f_hi + np.arange(nchans, dtype=np.float64) * foff


def band_freqs(f_top: float, f_bottom: float, nchans: int) -> np.ndarray:
    """A band written as 'f_top -> f_bottom' split into nchans channels of
    width (f_bottom - f_top)/nchans, channel 0 at f_top."""
    return channel_freqs(f_top, (f_bottom - f_top) / nchans, nchans)


def sky_delay_samples(dm: float, freqs: np.ndarray, tsamp: float) -> np.ndarray:
    """Arrival sample of a dispersed impulse in each channel, relative to its
    arrival at the highest frequency of the band: the cold-plasma delay
    K*DM*(f^-2 - f_top^-2) in seconds, rounded half-up to native samples."""
    f_top = float(np.max(freqs))
    delay_s = K_DISP * dm * (np.power(freqs, -2.0) - f_top ** -2.0)
    return np.floor(delay_s / tsamp + 0.5).astype(np.int64)


@dataclass(frozen=True)
class Pulse:
    dm: float      # pc cm^-3
    t0: int        # arrival sample at the top of the band
    width: int     # samples
    amp: float     # added to every sample the pulse covers


# --------------------------------------------------------------------------
# Filterbanks
# --------------------------------------------------------------------------

def _add_pulses(block: np.ndarray, c0: int, freqs: np.ndarray, tsamp: float,
                pulses) -> None:
    nb, nsamp = block.shape
    for p in pulses:
        delays = sky_delay_samples(p.dm, freqs, tsamp)[c0:c0 + nb]
        for k in range(p.width):
            t = p.t0 + delays + k
            ok = t < nsamp
            block[np.nonzero(ok)[0], t[ok]] += p.amp


def filterbank_u8(seed: int, freqs: np.ndarray, tsamp: float, nsamp: int,
                  pulses=(), mean: float = 128.0, sd: float = 16.0,
                  threads: int | None = None) -> np.ndarray:
    """uint8 filterbank [nchans][nsamp], channel-major.

    Noise is rint(N(mean, sd)) (half-to-even), the integer pulse amplitude is
    added, then the result is clipped once to [0, 255]."""
    nchans = len(freqs)
    out = np.empty((nchans, nsamp), dtype=np.uint8)
    nblk = (nchans + NOISE_BLOCK - 1) // NOISE_BLOCK
    kids = _substreams(seed)["noise"].spawn(nblk)

    def work(b):
        c0 = b * NOISE_BLOCK
        c1 = min(nchans, c0 + NOISE_BLOCK)
        rng = np.random.default_rng(kids[b])
        z = rng.standard_normal((c1 - c0, nsamp), dtype=np.float32)
        v = np.rint(z * np.float32(sd) + np.float32(mean)).astype(np.int16)
        _add_pulses(v, c0, freqs, tsamp, pulses)
        np.clip(v, 0, 255, out=v)
        out[c0:c1] = v

    with ThreadPoolExecutor(threads or _threads()) as ex:
        list(ex.map(work, range(nblk)))
    return out


def filterbank_u8_device(seed: int, freqs: np.ndarray, tsamp: float, nsamp: int, pulses=(),
                         mean: float = 128.0, sd: float = 16.0, device="cuda"):
    """The uint8 filterbank recipe of filterbank_u8 drawn on the GPU with
    torch's seeded generator (a different noise stream than the numpy one,
    for workloads too large to draw on the host): rint(N(mean, sd)) noise,
    integer pulses added, one clip to [0, 255]."""
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    nch = len(freqs)
    out = torch.empty((nch, nsamp), dtype=torch.uint8, device=device)
    step = max(1, (1 << 26) // max(1, nsamp))          # channels per chunk
    rows_all = [(p, sky_delay_samples(p.dm, freqs, tsamp)) for p in pulses]
    for c0 in range(0, nch, step):
        c1 = min(nch, c0 + step)
        z = torch.randn((c1 - c0, nsamp), generator=g, device=device, dtype=torch.float32)
        v = torch.round(z * sd + mean).to(torch.int16)
        for p, delays in rows_all:
            amp = int(p.amp)
            for k in range(p.width):
                t = p.t0 + delays[c0:c1] + k
                ok = np.nonzero(t < nsamp)[0]
                if ok.size:
                    ri = torch.from_numpy(ok).to(device)
                    ti = torch.from_numpy(t[ok]).to(device)
                    v[ri, ti] += amp
        out[c0:c1] = v.clamp_(0, 255).to(torch.uint8)
    return out


def filterbank_f32(seed: int, nchans: int, nsamp: int,
                   threads: int | None = None) -> np.ndarray:
    """float32 filterbank [nchans][nsamp] of N(0, 1) samples."""
    out = np.empty((nchans, nsamp), dtype=np.float32)
    nblk = (nchans + NOISE_BLOCK - 1) // NOISE_BLOCK
    kids = _substreams(seed)["noise"].spawn(nblk)

    def work(b):
        c0 = b * NOISE_BLOCK
        c1 = min(nchans, c0 + NOISE_BLOCK)
        rng = np.random.default_rng(kids[b])
        out[c0:c1] = rng.standard_normal((c1 - c0, nsamp), dtype=np.float32)

    with ThreadPoolExecutor(threads or _threads()) as ex:
        list(ex.map(work, range(nblk)))
    return out


def pulse_image(freqs: np.ndarray, tsamp: float, nsamp: int, pulses) -> np.ndarray:
    """The dispersed pulses alone, without noise or clipping, as int32
    [nchans][nsamp] (for closed-form and linearity checks)."""
    img = np.zeros((len(freqs), nsamp), dtype=np.int32)
    _add_pulses(img, 0, freqs, tsamp, [Pulse(p.dm, p.t0, p.width, int(p.amp)) for p in pulses])
    return img


def noise_only_u8(seed: int, freqs: np.ndarray, tsamp: float, nsamp: int,
                  threads: int | None = None) -> np.ndarray:
    """The same filterbank as filterbank_u8 with no pulse added."""
    return filterbank_u8(seed, freqs, tsamp, nsamp, (), threads=threads)


def gaussian(seed: int, shape, stream: str = "grad") -> np.ndarray:
    """float32 N(0, 1) array of the given shape from one named substream
    (used for output-gradient seeds and similar)."""
    rng = np.random.default_rng(_substreams(seed)[stream])
    return rng.standard_normal(shape, dtype=np.float32)


def random_u8(seed: int, shape) -> np.ndarray:
    """Uniform uint8 bytes over [0, 255] (for edge-case parity tests)."""
    rng = np.random.default_rng(_substreams(seed)["noise"])
    return rng.integers(0, 256, size=shape, dtype=np.uint8)


# --------------------------------------------------------------------------
# Workload descriptions
# --------------------------------------------------------------------------

@dataclass
class Workload:
    name: str
    freqs: np.ndarray
    tsamp: float
    nsamp: int
    ranges: list               # [(dm_lo, dm_hi, dm_step, downsample), ...]
    dtype: str                 # "u8" or "f32"
    seed: int
    pulses: list = field(default_factory=list)

    @property
    def nchans(self) -> int:
        return len(self.freqs)

    def make_input(self, threads: int | None = None) -> np.ndarray:
        if self.dtype == "u8":
            return filterbank_u8(self.seed, self.freqs, self.tsamp, self.nsamp,
                                 self.pulses, threads=threads)
        return filterbank_f32(self.seed, self.nchans, self.nsamp, threads=threads)


# The DM plan of the SKA-like single beam: five ranges with growing step and
# time downsampling.
SKA_RANGES = [
    (0.0, 150.0, 0.1, 1),
    (150.0, 300.0, 0.2, 2),
    (300.0, 500.0, 0.5, 4),
    (500.0, 1000.0, 1.0, 8),
    (1000.0, 2000.0, 2.0, 16),
]


def ska_ranges_upto(dm_max: float) -> list:
    return [r for r in SKA_RANGES if r[1] <= dm_max]


def _slot_pulses(rng, n: int, nsamp: int, guard: int, dm_lo: float,
                 dm_hi: float, wmin: int, wmax: int, amp: float) -> list:
    """n pulses with random DM and width; the usable span [0, nsamp-guard) is
    cut into n equal slots and each t0 falls in the first half of its slot,
    so the dispersed sweeps never overlap."""
    span = nsamp - guard
    slot = span // n
    out = []
    for i in range(n):
        dm = float(rng.uniform(dm_lo, dm_hi))
        w = int(rng.integers(wmin, wmax + 1))
        t0 = i * slot + int(rng.integers(0, max(1, slot // 2)))
        out.append(Pulse(dm=dm, t0=t0, width=w, amp=amp))
    return out


def tiny() -> Workload:
    """128 channels uint8, 1500 MHz top, channel width -2.34375 MHz, tsamp
    256 us, 65536 samples, DM 0..99 step 1; one pulse at DM 50, width 4,
    +48 counts, with its arrival drawn in [0, 65135)."""
    seed = 0
    freqs = channel_freqs(1500.0, -2.34375, 128)
    rng = np.random.default_rng(_substreams(seed)["pulses"])
    t0 = int(rng.integers(0, 65139 - 4))
    return Workload("tiny-128ch-u8", freqs, 256e-6, 65536, [(0.0, 100.0, 1.0, 1)],
                    "u8", seed, [Pulse(50.0, t0, 4, 48)])


def ska_single_beam(nsamp: int = 1 << 18, nchans: int = 4096) -> Workload:
    """4096 channels uint8 over 1670 -> 1370 MHz, tsamp 64 us, 2^18 samples,
    the five-range SKA-like plan up to DM 2000, five pulses with DM in
    [0, 2000), width 1-64 samples and amplitude 16 counts."""
    seed = 1
    freqs = band_freqs(1670.0, 1370.0, nchans)
    tsamp = 64e-6
    guard = int(sky_delay_samples(2000.0, freqs, tsamp).max()) + 64
    rng = np.random.default_rng(_substreams(seed)["pulses"])
    pulses = _slot_pulses(rng, 5, nsamp, guard, 0.0, 2000.0, 1, 64, 16)
    return Workload("ska-4096ch-u8-5ranges", freqs, tsamp, nsamp, list(SKA_RANGES),
                    "u8", seed, pulses)


def differentiable() -> Workload:
    """1024 channels float32 N(0,1), 1500 -> 1200 MHz, tsamp 128 us, 2^16
    samples, DM 0..511 step 1."""
    return Workload("diff-1024ch-f32", band_freqs(1500.0, 1200.0, 1024), 128e-6,
                    1 << 16, [(0.0, 512.0, 1.0, 1)], "f32", 2)


def batched_beams(nbeams: int = 64, seed: int = 3) -> list:
    """Beams of uneven shape: channel count from {1024, 2048, 4096}, length
    uniform in [2^16, 2^18], tsamp 64 or 128 us, DM max from {500, 1000,
    2000} with the SKA-like plan truncated there, two pulses per beam."""
    rng = np.random.default_rng(_substreams(seed)["beams"])
    beams = []
    for b in range(nbeams):
        nch = int(rng.choice([1024, 2048, 4096]))
        nsamp = int(rng.integers(1 << 16, (1 << 18) + 1))
        tsamp = float(rng.choice([64e-6, 128e-6]))
        dm_max = float(rng.choice([500.0, 1000.0, 2000.0]))
        freqs = band_freqs(1670.0, 1370.0, nch)
        guard = int(sky_delay_samples(dm_max, freqs, tsamp).max()) + 64
        pulses = _slot_pulses(rng, 2, nsamp, guard, 0.0, dm_max, 1, 64, 16)
        beams.append(Workload(f"beam{b}-{nch}ch", freqs, tsamp, nsamp,
                              ska_ranges_upto(dm_max), "u8", 1000 * seed + b, pulses))
    return beams


def batched_differentiable(nbeams: int = 32, nsamp: int = 1 << 17) -> list:
    """Beams of 4096 channels float32, 1670 -> 1370 MHz, tsamp 64 us, DM
    0..999 step 1."""
    freqs = band_freqs(1670.0, 1370.0, 4096)
    return [Workload(f"diffbeam{b}", freqs, 64e-6, nsamp, [(0.0, 1000.0, 1.0, 1)],
                     "f32", 4000 + b) for b in range(nbeams)]
