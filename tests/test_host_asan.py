"""Host code under AddressSanitizer and UBSan (CPU only): the packing of the
caller's [nv][nc] coefficient arrays into the kernels' launch arguments,
for every nv = 1..8 and nc = 1..8, with caller arrays of exactly 2 nv nc
doubles (tests/native/coef_pack_check.cpp)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_coef_packing_under_asan(tmp_path):
    exe = str(tmp_path / "coef_pack_check")
    src = os.path.join(ROOT, "tests", "native", "coef_pack_check.cpp")
    inc = os.path.join(ROOT, "paper_2005_13498_amd", "csrc")
    subprocess.run(["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                    "-I", inc, src, "-o", exe], check=True)
    r = subprocess.run([exe], capture_output=True, text=True, env={**os.environ, "ASAN_OPTIONS": "detect_leaks=1"})
    assert r.returncode == 0, r.stdout + r.stderr
    assert "coef_pack ok" in r.stdout
