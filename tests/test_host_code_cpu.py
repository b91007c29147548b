"""The library's host code (validation, layout, tile lists, checkpoints, the
adjoint's segment bookkeeping) run on the CPU against a stub HIP runtime whose
kernel launches check every tile and address range they would touch; built
with the C++ library's bounds assertions. Regression cover for host-side
indexing mistakes, such as reading per-grid tables with the padding entries
(grid -1) of the die-ordered tile lists."""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests", "host_sim")


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_host_code_paths_stay_in_bounds(tmp_path):
    lib = str(tmp_path / "libhostsim.so")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fPIC", "-shared", "-D_GLIBCXX_ASSERTIONS",
           "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include", "-I" + os.path.join(ROOT, "include"),
           "-I" + os.path.join(ROOT, "paper_2009_06404_amd", "csrc"), "-Wno-unused-result",
           os.path.join(ROOT, "paper_2009_06404_amd", "csrc", "lbm_api.cpp"),
           os.path.join(ROOT, "paper_2009_06404_amd", "csrc", "lbm_stability.cpp"),
           os.path.join(HERE, "stub.cpp"), "-o", lib]
    subprocess.run(cmd, check=True)
    r = subprocess.run([sys.executable, os.path.join(HERE, "drive.py"), lib],
                       capture_output=True, text=True, timeout=600)
    assert r.returncode == 0 and "ALL OK" in r.stdout, (r.returncode, r.stdout[-2000:],
                                                        r.stderr[-4000:])


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_three_dimensional_host_code_and_tile_split(tmp_path):
    """The 3-D host code (layout, tables, lean / general tile lists, stepping,
    fields, state copies) against the stub runtime: every tile inside the
    volume and its buffers, no lean tile that pulls a non-periodic face cell,
    lies within 9 sigma of a source or holds a receiver, and every cell
    written exactly once per step."""
    lib = str(tmp_path / "libhostsim3.so")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fPIC", "-shared", "-D_GLIBCXX_ASSERTIONS",
           "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include", "-I" + os.path.join(ROOT, "include"),
           "-I" + os.path.join(ROOT, "paper_2009_06404_amd", "csrc"), "-Wno-unused-result",
           os.path.join(ROOT, "paper_2009_06404_amd", "csrc", "lbm_api.cpp"),
           os.path.join(ROOT, "paper_2009_06404_amd", "csrc", "lbm3d_api.cpp"),
           os.path.join(ROOT, "paper_2009_06404_amd", "csrc", "lbm_stability.cpp"),
           os.path.join(ROOT, "paper_2009_06404_amd", "csrc", "lbm3d_stability.cpp"),
           os.path.join(HERE, "stub.cpp"), os.path.join(HERE, "stub3.cpp"), "-o", lib]
    subprocess.run(cmd, check=True)
    r = subprocess.run([sys.executable, os.path.join(HERE, "drive3.py"), lib],
                       capture_output=True, text=True, timeout=600)
    print(r.stdout[-500:])
    assert r.returncode == 0 and "ALL OK" in r.stdout, (r.returncode, r.stdout[-2000:],
                                                        r.stderr[-4000:])
