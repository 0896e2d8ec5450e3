"""The engine's division by a field's invariant divisors (a multiply and a
shift with magic numbers from the host) against plain integer division, on
the host: compiled with hipcc from the library's own header."""
import os
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_2601_01787_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not found")
def test_fast_division_is_exact(tmp_path):
    exe = str(tmp_path / "fastdiv_check")
    subprocess.run([HIPCC, "-O2", "-std=c++17", "-I", CSRC,
                    os.path.join(HERE, "native", "fastdiv_check.hip"), "-o", exe],
                   check=True, capture_output=True)
    out = subprocess.run([exe], capture_output=True, text=True)
    assert out.returncode == 0, out.stdout + out.stderr
    assert "bad 0" in out.stdout
