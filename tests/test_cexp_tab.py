"""The near-field sweep's complex exponential (table reductions and short
Taylor polynomials, csrc/cexp_tab.h), compiled for the host with hipcc and
checked against long-double exp, cos and sin: relative error below 1e-15 over
the argument ranges the sweep produces, zero and infinity at the ends."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_1902_08250_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not found")
def test_cexp_tab_host(tmp_path):
    exe = str(tmp_path / "cexp_tab_check")
    cmd = [HIPCC, "-x", "hip", "--cuda-host-only", "-O2", "-std=c++17", "-I" + CSRC,
           os.path.join(HERE, "native", "cexp_tab_check.cpp"), "-o", exe]
    subprocess.run(cmd, check=True, capture_output=True, timeout=300)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    print(r.stdout)
    assert r.returncode == 0, r.stdout + r.stderr
