"""The LDS tile that the host allots to a brick's detector footprint must
hold every tap the kernels read (Alg. 3's four taps of every voxel, at the
coordinates of Eq. 3 and Theorems 1-3 computed as the kernels do). A short
tile would give wrong values without any fault, so this is checked on the
CPU: tests/tile_bounds_check.cpp builds the kernels' brick setup and FP32
column arithmetic for the host and walks seeded random geometries (volume
and detector shapes, pitches, principal-point shifts with and without a
pixel-aligned mirror, magnifications from 0.3 to 3 pixels per voxel, view
angles anywhere on the circle, mirrored and plain runs)."""
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"


@pytest.fixture(scope="module")
def checker(tmp_path_factory):
    exe = tmp_path_factory.mktemp("tiles") / "tile_bounds_check"
    cmd = [HIPCC, "-std=c++17", "-O2", "--offload-arch=gfx950", "--cuda-host-only",
           "-x", "hip", os.path.join(ROOT, "tests", "tile_bounds_check.cpp"),
           "-x", "c++", os.path.join(ROOT, "paper_1909_02724_amd", "csrc", "tiles.cpp"),
           "-o", str(exe)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    return exe


@pytest.mark.parametrize("seed", [1, 20240917])
def test_every_tap_inside_the_tile(checker, seed):
    out = subprocess.run([str(checker), str(seed), "2000"], capture_output=True, text=True,
                         check=True).stdout
    rows = {}
    for line in out.splitlines():
        kind, *fields = line.split()
        rows[kind] = {k: int(v) for k, v in (f.split("=") for f in fields)}
    print(out)
    for kind in ("mirror", "plain"):
        s = rows[kind]
        assert s["tiled"] >= 200, s            # enough geometries take the LDS path
        assert s["columns"] >= 10_000_000, s
        assert s["neg"] == 0, s                # coordinates stay above the tile origin
        assert s["col_viol"] == 0 and s["row_viol"] == 0, s
        assert s["min_col_slack"] >= 1 and s["min_row_slack"] >= 1, s
