"""The sub-band kernel's LDS schedule and index math, emulated on the CPU.

tests/emu/sb_schedule.cpp replays k_dedisp_u8_sb's stages on the host
tables of variant-3 plans (built by the library's own plan code): it
bounds-checks every LDS and global index, checks that every needed LDS read
sees a word written for its stage and landed behind a wait and a barrier,
that no word is written and read between the same two barriers, and that
every output equals the direct sum over the shift table.  Small plans at
every DM tile, including one-channel and ragged bands, large downsampling
and one-sub-band stages, then random plans.  No GPU.
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
    exe = str(tmp_path_factory.mktemp("sb") / "sb_schedule")
    subprocess.run(["g++", "-O2", "-std=c++17", "-pthread", "-I", CSRC,
                    "-I", os.path.join(ROOT, "include"),
                    os.path.join(HERE, "emu", "sb_schedule.cpp"),
                    os.path.join(CSRC, "plan.cpp"), "-o", exe], check=True)
    return exe


def test_small_plans_every_tile(emulator):
    r = subprocess.run([emulator, "small", "3"], capture_output=True, text=True, timeout=600)
    assert r.returncode == 0 and "FAIL" not in r.stdout, r.stdout[-3000:]
    checked = [int(m) for m in re.findall(r"checked (\d+) outputs, 0 mismatches, fails 0", r.stdout)]
    # plans that do not fit the LDS at a tile are skipped; most fit
    assert len(checked) >= 30 and sum(checked) > 10_000_000, r.stdout[-3000:]
    # rows with every count of odd-aligned channels occurred
    hist = [int(v) for v in re.search(r"rows by odd-aligned channels:([ \d]+)", r.stdout).group(1).split()]
    assert len(hist) == 9 and all(h > 0 for h in hist), hist


def test_random_plans(emulator):
    """36 random plans (band, possibly permuted; sampling; length; one to
    three ranges of random step and downsample up to 16) over every DM tile
    and time tile; those whose patterns do not fit the LDS are skipped."""
    r = subprocess.run([emulator, "random", "1"], capture_output=True, text=True, timeout=600)
    assert r.returncode == 0 and "FAIL" not in r.stdout, r.stdout[-3000:]
    checked = [int(m) for m in re.findall(r"checked (\d+) outputs, 0 mismatches, fails 0", r.stdout)]
    assert len(checked) >= 24 and sum(checked) > 5_000_000, r.stdout[-3000:]
    assert len(re.findall(r"checked \d+ outputs", r.stdout)) == len(checked), r.stdout[-3000:]
