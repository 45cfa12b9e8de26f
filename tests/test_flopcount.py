"""The benchmark's algorithmic operation counts come from the operation counter.

paper_2402_02075_amd/csrc/flopcount.hip instantiates the face kernel's per-point physics on the
host with a scalar that counts every add, multiply, divide and transcendental call; this test
compiles it, runs it for both flux paths and both face kinds, and checks the constants bench.py
prices the face kernel with.
"""
import json
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def counter(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None or not os.path.isdir("/opt/rocm/include"):
        pytest.skip("needs g++ and the ROCm headers")
    exe = str(tmp_path_factory.mktemp("fc") / "flopcount")
    src = os.path.join(ROOT, "paper_2402_02075_amd", "csrc", "flopcount.hip")
    subprocess.run([gxx, "-O1", "-std=c++17", "-x", "c++", "-D__HIP_PLATFORM_AMD__", "-I", "/opt/rocm/include",
                    "-I", os.path.join(ROOT, "include"), src, "-o", exe], check=True, capture_output=True)

    def run(ngp, path):
        r = subprocess.run([exe, str(ngp), path], check=True, capture_output=True, text=True)
        return json.loads(r.stdout)
    return run


@pytest.mark.parametrize("path", ["inviscid", "viscous"])
def test_bench_constants_match_the_counter(counter, path):
    import bench
    for ngp in (3, 4):
        c = counter(ngp, path)
        assert c["face_sum_per_point"] == pytest.approx(bench.FACE_SUM_OPS * (ngp - 1) / ngp)
        assert c["flops_per_point"] - c["face_sum_per_point"] == pytest.approx(bench.FLOPS_PER_GP[path])
    # per launch: each face's points carry the per-point count plus the face sums
    assert bench.face_flops_per_launch(path, 7, 2) == pytest.approx(
        3 * counter(3, path)["flops_per_point"] + 4 * counter(4, path)["flops_per_point"])
