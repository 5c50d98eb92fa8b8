"""The per-lane node update's fused passes against the separate passes they
replace, built for the CPU.

tests/host/pwl_fused_check.cpp compiles bt_pwl.hpp with g++ and checks, on
seeded random functions with collinear runs, lines and slopes one ulp apart:
MERGE with SCALE and the scaled CANON in one pass (merge_scale) against
MERGE, SCALE, CANON; CLIP's clamp with its CANON against the two passes;
the envelope's sweep read back with CANON (sweep_a) and the mirror image of
the second sweep with CANON (mirror_canon_raw) against reversal, slope shift,
CANON and mirror written out from their definitions.  Counts and every stored
number must agree bit for bit, and the cases must reach the branches where
CANON drops points after scaling or leaves a line."""
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "host", "pwl_fused_check.cpp")
CSRC = os.path.join(ROOT, "paper_1110_2477_amd", "csrc")
ROCM_INC = "/opt/rocm/include"


def test_fused_passes_match_the_separate_passes(tmp_path):
    if shutil.which("g++") is None or not os.path.isdir(ROCM_INC):
        pytest.skip("g++ or the ROCm headers are not available")
    exe = str(tmp_path / "pwl_fused_check")
    cmd = ["g++", "-O2", "-std=c++17", "-D__HIP_PLATFORM_AMD__", "-I" + ROCM_INC, "-I" + CSRC, "-o", exe, SRC]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    r = subprocess.run([exe, "20000"], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr[-2000:]
    m = re.match(r"ok (\d+) merges (\d+) clips (\d+) sweeps (\d+) scaled-canon-drops (\d+) lines (\d+) "
                 r"sweep-canon-drops (\d+)", r.stdout)
    assert m, r.stdout
    cases, merges, clips, sweeps, drops, lines, sdrops = map(int, m.groups())
    assert cases == 20000 and merges == 2 * cases and clips == cases and sweeps == cases
    # not vacuous: scaling merges distinct slopes, lines occur, sweeps drop points
    assert drops > 100 and lines > 100 and sdrops > 100
