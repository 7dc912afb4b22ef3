"""Host logic of the contraction planner: every GEMM operand and output
address map of every device program is an in-bounds bijection onto its
tensor or pack buffer (tests/native/planner_check.cpp, built here against
libscc.so; no GPU needed)."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
PKG = os.path.join(ROOT, "paper_2403_01007_amd")


@pytest.fixture(scope="module")
def checker(tmp_path_factory):
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    if not os.path.exists(os.path.join(PKG, "libscc.so")):
        pytest.skip("libscc.so not built")
    if not shutil.which(hipcc) and not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    exe = str(tmp_path_factory.mktemp("planner") / "planner_check")
    cmd = [hipcc, "-O1", "-std=c++17", os.path.join(HERE, "native", "planner_check.cpp"), "-L", PKG, "-lscc",
           f"-Wl,-rpath,{PKG}", "-o", exe]
    subprocess.run(cmd, check=True, capture_output=True, timeout=600)
    return exe


@pytest.mark.parametrize("dims", [(2, 4, 12, 3), (4, 12, 40, 3), (5, 19, 60, 3), (3, 9, 20, 2),
                                  (10, 90, 300, 3)],  # the o10v90 workload bench.py times (about a minute)
                         ids=["o2v4", "o4v12", "o5v19", "o3v9", "o10v90"])
def test_gemm_address_maps_are_bijections(checker, dims):
    r = subprocess.run([checker] + [str(x) for x in dims], capture_output=True, text=True, timeout=600)
    print(r.stdout)
    assert r.returncode == 0, r.stdout + r.stderr
    assert r.stdout.startswith("ok:")
