"""Host ordering of sas_peaks: the radix sort on mixed-radix keys (and its
comparison fallback for ranges beyond 64 bits) against a plain stable sort
with the field comparison.  Compiled with g++; no GPU."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not found")
def test_candidate_order(tmp_path):
    exe = str(tmp_path / "peaks_sort_check")
    subprocess.run(["g++", "-O2", "-std=c++17", "-Wall", "-o", exe,
                    os.path.join(HERE, "peaks_sort_check.cpp")], check=True)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "0 mismatches" in r.stdout
