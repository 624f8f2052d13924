"""Writes the stored expected values under tests/golden/.

Every value is computed by the oracle's exact-rational reading of the delay
(oracle.dedisp.shift_exact); nothing here comes from the HIP library.

    python tests/golden/make_golden.py
"""
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

import synth  # noqa: E402
from oracle import dedisp as O  # noqa: E402


def near_ties(path, tol=1e-6):
    """Shift-table entries of the reference workloads whose FP64 delay lies
    within tol of a rounding tie, with the exact-rational rounded value."""
    wls = [synth.tiny(), synth.ska_single_beam(), synth.differentiable(),
           synth.batched_differentiable(1)[0]]
    rows = []
    for w in wls:
        f_ref = float(w.freqs.max())
        for r, (lo, hi, step, ds) in enumerate(w.ranges):
            dms = O.range_dms(lo, hi, step)
            x = O.shift_x_table(w.freqs, w.tsamp, dms, ds)
            frac = x - np.floor(x)
            d_i, c_i = np.nonzero(np.abs(frac - 0.5) < tol)
            for d, c in zip(d_i, c_i):
                s = O.shift_exact(w.freqs[c], f_ref, w.tsamp, dms[d], ds)
                xe = O.shift_exact_x(w.freqs[c], f_ref, w.tsamp, dms[d], ds)
                rows.append((w.name, r, int(d), int(c), repr(float(dms[d])),
                             repr(float(w.freqs[c])), s, float(xe - int(xe))))
    with open(path, "w") as f:
        f.write("# Shift-table entries of the reference workloads whose delay x lies within\n"
                "# 1e-6 of a half-integer, with floor(x + 1/2) evaluated in exact rational\n"
                "# arithmetic from the FP64 inputs.  Written by tests/golden/make_golden.py.\n"
                "# workload range dm_index channel dm freq_mhz exact_shift exact_frac\n")
        for row in rows:
            f.write(" ".join(str(v) for v in row) + "\n")
    return len(rows)


if __name__ == "__main__":
    n = near_ties(os.path.join(HERE, "shift_near_ties.txt"))
    print("near ties:", n)
