"""CPU check of the split of a mixed-size SGEMM launch over the 8 XCDs
(csrc/gemm_balance.hpp, used by csrc/sgemm.hip): runs of equal work, and the
kernel's index walk over the balanced grid visits every tile exactly once
(tests/cpp/test_gemm_balance.cpp)."""

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_xcd_runs_cover_every_tile_once_with_equal_work(tmp_path):
    exe = str(tmp_path / "test_gemm_balance")
    subprocess.run(["g++", "-O2", "-std=c++17", "-Wall", "-Werror", f"-I{ROOT}/paper_1511_07658_amd/csrc",
                    f"{ROOT}/tests/cpp/test_gemm_balance.cpp", "-o", exe], check=True)
    p = subprocess.run([exe], stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True, timeout=120)
    assert p.returncode == 0, p.stdout[-3000:]
    assert p.stdout.strip().endswith("ok: 0 failures"), p.stdout[-3000:]
