"""The plan cache's pin accounting on the CPU: tests/native/plan_cache_check.cpp
drives the cache bookkeeping (paper_1702_08159_amd/csrc/plan_cache.hpp, the
same header the runtime builds) through calls that leave by every exit path,
evictions under pins and `captured` marks, and shutdown."""
import os
import shutil
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1702_08159_amd", "csrc")
SRC = os.path.join(ROOT, "tests", "native", "plan_cache_check.cpp")


@pytest.mark.skipif(shutil.which("g++") is None, reason="no host C++ compiler")
def test_plan_cache_pin_accounting():
    with tempfile.TemporaryDirectory() as tmp:
        exe = os.path.join(tmp, "plan_cache_check")
        subprocess.run(["g++", "-std=c++17", "-O1", "-Wall", "-Werror", "-I" + CSRC, SRC, "-o", exe,
                        "-pthread"], check=True)
        res = subprocess.run([exe], capture_output=True, text=True)
    assert res.returncode == 0, res.stdout + res.stderr
    assert "passed" in res.stdout
