"""Host check of the solvers' subspace eigensolvers (tests/native/eig_check.cpp,
compiled here with the host compiler; no GPU): the real double-shift QR
agrees with the complex single-shift QR on random nonsymmetric matrices with
real and complex spectra, and inverse iteration gives eigenvectors with small
residuals."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


def test_subspace_eigensolvers(tmp_path):
    cxx = shutil.which("g++")
    if not cxx:
        pytest.skip("no host C++ compiler")
    exe = str(tmp_path / "eig_check")
    subprocess.run([cxx, "-O2", "-std=c++17", os.path.join(HERE, "native", "eig_check.cpp"), "-o", exe],
                   check=True, capture_output=True, timeout=300)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    print(r.stdout)
    assert r.returncode == 0, r.stdout + r.stderr
    assert r.stdout.startswith("ok:")
