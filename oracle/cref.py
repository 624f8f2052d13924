"""ctypes front of the plain C oracle (``oracle/dedisp_ref.c``).

TEST INFRASTRUCTURE ONLY: used by tests, the smoke check and the benchmark's
CPU-baseline leg; the product never loads it.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(_HERE, "dedisp_ref.c")
LIB = os.path.join(_HERE, "libdedisp_ref.so")

_lib = None


def build() -> str:
    """Compile the C oracle with gcc (plain -O3, OpenMP, no FMA contraction so
    its FP64 shift table follows the written operation order)."""
    cmd = ["gcc", "-O3", "-std=c11", "-fopenmp", "-ffp-contract=off", "-shared",
           "-fPIC", "-o", LIB + ".tmp", SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        L = ctypes.CDLL(LIB)
        P = ctypes.c_void_p
        i32, i64, f64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_double
        L.oracle_plan_sizes.argtypes = [P, i32, f64, i64, P, i32, P, P]
        L.oracle_range_shifts.argtypes = [P, i32, f64, P, P]
        L.oracle_dedisperse_u8_rows.argtypes = [P, i32, i64, P, f64, P, i32, i32, P, i32]
        L.oracle_dedisperse_u8.argtypes = [P, i32, i64, P, f64, P, i32, P, i64, i32]
        L.oracle_dedisperse_f32.argtypes = [P, i32, i64, P, f64, P, i32, P, P, i64, i32]
        L.oracle_adjoint_f32.argtypes = [P, i32, i64, P, f64, P, i32, P, P, P, P, i32]
        for f in ("oracle_plan_sizes", "oracle_range_shifts", "oracle_dedisperse_u8_rows",
                  "oracle_dedisperse_u8", "oracle_dedisperse_f32", "oracle_adjoint_f32",
                  "oracle_max_threads"):
            getattr(L, f).restype = ctypes.c_int
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _ranges(ranges) -> np.ndarray:
    return np.ascontiguousarray(np.array(ranges, dtype=np.float64).reshape(-1, 4))


def plan_sizes(freqs, tsamp, nsamp, ranges):
    rg = _ranges(ranges)
    f = np.ascontiguousarray(freqs, dtype=np.float64)
    nd = np.zeros(len(rg), dtype=np.int32)
    no = np.zeros(len(rg), dtype=np.int64)
    rc = lib().oracle_plan_sizes(_ptr(f), len(f), tsamp, nsamp, _ptr(rg), len(rg),
                                 _ptr(nd), _ptr(no))
    if rc:
        raise ValueError(f"oracle_plan_sizes failed ({rc})")
    return nd, no


def range_shifts(freqs, tsamp, rng):
    rg = _ranges([rng])
    f = np.ascontiguousarray(freqs, dtype=np.float64)
    nd = int(np.floor((rg[0, 1] - rg[0, 0]) / rg[0, 2] + 0.5))
    s = np.zeros((nd, len(f)), dtype=np.int32)
    if lib().oracle_range_shifts(_ptr(f), len(f), tsamp, _ptr(rg), _ptr(s)):
        raise ValueError("oracle_range_shifts failed")
    return s


def dedisperse_u8(x: np.ndarray, freqs, tsamp, ranges, threads: int = 0) -> np.ndarray:
    x = np.ascontiguousarray(x, dtype=np.uint8)
    nd, no = plan_sizes(freqs, tsamp, x.shape[1], ranges)
    if (no <= 0).any():
        raise ValueError("empty range")
    out = np.zeros(int((nd.astype(np.int64) * no).sum()), dtype=np.int32)
    rg = _ranges(ranges)
    f = np.ascontiguousarray(freqs, dtype=np.float64)
    rc = lib().oracle_dedisperse_u8(_ptr(x), x.shape[0], x.shape[1], _ptr(f), tsamp,
                                    _ptr(rg), len(rg), _ptr(out), out.size, threads)
    if rc:
        raise ValueError(f"oracle_dedisperse_u8 failed ({rc})")
    return out


def dedisperse_u8_rows(x: np.ndarray, freqs, tsamp, rng, d_begin, d_end, nout,
                       threads: int = 0) -> np.ndarray:
    x = np.ascontiguousarray(x, dtype=np.uint8)
    out = np.zeros((d_end - d_begin, nout), dtype=np.int32)
    rg = _ranges([rng])
    f = np.ascontiguousarray(freqs, dtype=np.float64)
    rc = lib().oracle_dedisperse_u8_rows(_ptr(x), x.shape[0], x.shape[1], _ptr(f), tsamp,
                                         _ptr(rg), d_begin, d_end, _ptr(out), threads)
    if rc:
        raise ValueError(f"oracle_dedisperse_u8_rows failed ({rc})")
    return out


def dedisperse_f32(x: np.ndarray, freqs, tsamp, ranges, weights=None,
                   threads: int = 0) -> np.ndarray:
    x = np.ascontiguousarray(x, dtype=np.float32)
    nd, no = plan_sizes(freqs, tsamp, x.shape[1], ranges)
    if (no <= 0).any():
        raise ValueError("empty range")
    out = np.zeros(int((nd.astype(np.int64) * no).sum()), dtype=np.float64)
    rg = _ranges(ranges)
    f = np.ascontiguousarray(freqs, dtype=np.float64)
    w = None if weights is None else np.ascontiguousarray(weights, dtype=np.float32)
    rc = lib().oracle_dedisperse_f32(_ptr(x), x.shape[0], x.shape[1], _ptr(f), tsamp,
                                     _ptr(rg), len(rg), None if w is None else _ptr(w),
                                     _ptr(out), out.size, threads)
    if rc:
        raise ValueError(f"oracle_dedisperse_f32 failed ({rc})")
    return out


def adjoint_f32(x: np.ndarray, freqs, tsamp, ranges, g: np.ndarray, weights=None,
                threads: int = 0):
    """(dX, dw) in double for the concatenated output gradient g."""
    x = np.ascontiguousarray(x, dtype=np.float32)
    g = np.ascontiguousarray(g, dtype=np.float64)
    rg = _ranges(ranges)
    f = np.ascontiguousarray(freqs, dtype=np.float64)
    w = None if weights is None else np.ascontiguousarray(weights, dtype=np.float32)
    dX = np.zeros(x.shape, dtype=np.float64)
    dw = np.zeros(x.shape[0], dtype=np.float64)
    rc = lib().oracle_adjoint_f32(_ptr(x), x.shape[0], x.shape[1], _ptr(f), tsamp, _ptr(rg),
                                  len(rg), None if w is None else _ptr(w), _ptr(g), _ptr(dX),
                                  _ptr(dw), threads)
    if rc:
        raise ValueError(f"oracle_adjoint_f32 failed ({rc})")
    return dX, dw


def max_threads() -> int:
    return int(lib().oracle_max_threads())
