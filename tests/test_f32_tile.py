"""The float32 shift-and-sum tile's index math, emulated on the CPU.

tests/emu/f32_tile.cpp follows k_shiftsum_f32 on the host tables of float32
plans (built by the library's own plan code), forward and adjoint problems:
every LDS and global index is bounds-checked; with sub-band reuse, the
level-1 jobs build each pattern row from its group's rows (reads inside
those rows' windows) and write only its slot; each stage row reaches every
output exactly once, directly or through a pattern row; every value a lane
uses comes from the row or pattern row its entry names; and every output of
lanes 0..62 equals the direct sum (integer-valued inputs, exact in any
order).  Plans with one channel, odd stages, permuted channels, two
downsamples, the 1024-channel differentiable band and a 4096-channel band,
with the default choice, direct sums only and sub-band reuse forced; then
24 random plans (band, sampling, length, one to three ranges of random step
and downsample, any strategy).  No GPU.
"""
import os
import re
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_1912_07704_amd", "csrc")


@pytest.fixture(scope="module")
def emulator(tmp_path_factory):
    if shutil.which("g++") is None:
        pytest.skip("g++ not available")
    exe = str(tmp_path_factory.mktemp("f32") / "f32_tile")
    subprocess.run(["g++", "-O2", "-std=c++17", "-pthread", "-I", CSRC,
                    "-I", os.path.join(ROOT, "include"),
                    os.path.join(HERE, "emu", "f32_tile.cpp"),
                    os.path.join(CSRC, "plan.cpp"), "-o", exe], check=True)
    return exe


def test_f32_tiles_forward_and_adjoint(emulator):
    r = subprocess.run([emulator], capture_output=True, text=True, timeout=600)
    assert r.returncode == 0 and "FAIL" not in r.stdout, r.stdout[-3000:]
    assert "plans 12 of 12, fails 0" in r.stdout, r.stdout[-3000:]
    fixed = r.stdout.split("plans 12 of 12")[0]
    checked = [int(a) + int(b) for a, b in re.findall(r"checked (\d+) \+ (\d+) outputs", fixed)]
    assert len(checked) == 17 and sum(checked) > 10_000_000, r.stdout[-3000:]
    # random plans (any strategy, one to three ranges): most must be accepted
    m = re.search(r"fuzz plans (\d+) of (\d+) accepted, fails 0", r.stdout)
    assert m and int(m.group(1)) >= int(m.group(2)) - 4, r.stdout[-3000:]
    # the forced sub-band plans (variant 3) build pattern rows in every problem
    for line in r.stdout.splitlines():
        if " sb] range" in line:
            assert re.search(r"patterns [1-9]\d*/[1-9]", line), line
