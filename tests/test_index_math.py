"""CPU guard of the GPU kernels' index arithmetic: builds tests/plane_index_check.cpp
(which uses the kernel's own index functions from plane_index.h) with the host compiler
and enumerates every global, LDS and solve index of the elastic plane pass on the
production workloads and the GPU test geometries."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

GEOMS = [
    # nx ny nz Mx My halo periodic shots
    (512, 512, 512, 64, 64, 12, 0, 1),     # 513^3 layered elastic workload
    (256, 256, 256, 64, 64, 10, 0, 2),     # 257^3 two-shot elastic workload
    (64, 64, 64, 32, 32, 10, 0, 2),
    (50, 50, 50, 16, 16, 6, 0, 2),
    (48, 40, 56, 16, 32, 8, 0, 2),
    (48, 48, 48, 24, 24, 10, 1, 2),
    (48, 48, 48, 24, 24, 8, 0, 2),
    (40, 40, 40, 8, 8, 6, 0, 2),
    (130, 70, 40, 64, 64, 12, 0, 2),
    (48, 48, 48, 24, 24, 6, 0, 1),         # lanes of a patch reaching past its taps
    (96, 96, 20, 64, 64, 12, 1, 1),        # periodic full tiles
]


@pytest.fixture(scope="module")
def checker(tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("idx") / "plane_index_check")
    subprocess.check_call(["g++", "-O2", "-std=c++17", "-I", os.path.join(ROOT, "paper_2301_05127_amd", "csrc"),
                           os.path.join(ROOT, "tests", "plane_index_check.cpp"), "-o", exe])
    return exe


@pytest.mark.parametrize("geom", GEOMS, ids=["x".join(map(str, g[:3])) + "M%d_h%d_p%d" % (g[3], g[5], g[6])
                                             for g in GEOMS])
def test_plane_pass_indices_in_bounds(checker, geom):
    out = subprocess.run([checker] + [str(v) for v in geom], capture_output=True, text=True)
    assert out.returncode == 0 and out.stdout.strip() == "ok", out.stdout
