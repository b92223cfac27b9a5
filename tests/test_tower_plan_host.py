"""The single-launch pyramid's host planner and the kernel's indexing,
replayed on the CPU (tests/host/tower_plan_check.hip) for 16 image sizes
with 2, 3, 8 and 12 levels and 8 tile shapes, against the oracle pyramid: every
level bit-exact, every pixel written once, no LDS access outside its
buffer, no weighted read of a byte the level above did not write."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_tower_plan_replayed_on_host(tmp_path):
    hipcc = "/opt/rocm/bin/hipcc" if os.path.exists("/opt/rocm/bin/hipcc") else shutil.which("hipcc")
    lib = os.path.join(ROOT, "paper_2410_04090_amd", "libvsfe.so")
    olib = os.path.join(ROOT, "oracle", "liboracle.so")
    if not hipcc or not os.path.exists(lib) or not os.path.exists(olib):
        pytest.skip("needs hipcc and the built library and oracle")
    exe = str(tmp_path / "tower_plan_check")
    src = os.path.join(ROOT, "tests", "host", "tower_plan_check.hip")
    cmd = [hipcc, "--offload-arch=gfx950", "-O1", "-std=c++17", "-Xclang", "-target-feature", "-Xclang",
           "-packed-fp32-ops", "-I", os.path.join(ROOT, "include"), "-I",
           os.path.join(ROOT, "paper_2410_04090_amd", "csrc"), src, "-o", exe,
           "-L", os.path.dirname(lib), "-lvsfe", "-L", os.path.dirname(olib), "-loracle",
           "-Wl,-rpath," + os.path.dirname(lib), "-Wl,-rpath," + os.path.dirname(olib)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    r = subprocess.run([exe], capture_output=True, text=True, timeout=600)
    print(r.stdout[-4000:])
    assert r.returncode == 0, r.stdout[-3000:]
    assert "fails: 0" in r.stdout
    # the default workloads' sizes are planned and pass
    for size in ("1241x376", "1920x1080", "752x480"):
        assert any(size in line and ": ok" in line for line in r.stdout.splitlines()), size
