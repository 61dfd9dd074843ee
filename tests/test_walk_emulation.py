"""The GPU ray walk (vg_walk.h, shared by the walk kernels) compiled for the
host and compared with the CPU oracle's walk ray by ray: random grids,
occupancy (bits, or stamp bytes), camera positions inside and outside the
grid, voxel-centre ties and zero direction components, both walk forms (for
wavefronts alone on a SIMD and for shared SIMDs) under random wavefront
votes.  Catches logic errors in the walk without a GPU; the GPU parity tests
cover the device build."""
import os
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


@pytest.fixture(scope="module")
def emu(tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("walk") / "walk_emu")
    subprocess.check_call(["g++", "-O2", "-std=c++17", "-ffp-contract=off", "-fno-fast-math",
                           "-Wall", "-o", exe, os.path.join(HERE, "walk_emu.cpp"),
                           "-x", "c", os.path.join(ROOT, "oracle", "vg_oracle.c"), "-lm"])
    return exe


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_host_build_of_walk_matches_oracle(emu, seed):
    out = subprocess.run([emu, "1500", str(seed)], capture_output=True, text=True, timeout=300)
    assert out.returncode == 0, out.stdout + out.stderr
    assert "mismatches 0" in out.stdout
