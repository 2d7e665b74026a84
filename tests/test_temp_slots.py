"""The rule that picks a cached temporary block, on the CPU:
tests/native/temp_slots_check.cpp drives the header the runtime builds
(paper_1702_08159_amd/csrc/temp_slots.hpp) through the preference order --
own stream and large enough, never used, own stream to grow, any free block
-- and checks that busy blocks are never taken."""
import os
import shutil
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1702_08159_amd", "csrc")
SRC = os.path.join(ROOT, "tests", "native", "temp_slots_check.cpp")


@pytest.mark.skipif(shutil.which("g++") is None, reason="no host C++ compiler")
def test_temp_slot_choice():
    with tempfile.TemporaryDirectory() as tmp:
        exe = os.path.join(tmp, "temp_slots_check")
        subprocess.run(["g++", "-std=c++17", "-O1", "-Wall", "-Werror", "-I" + CSRC, SRC, "-o", exe], check=True)
        res = subprocess.run([exe], capture_output=True, text=True)
    assert res.returncode == 0, res.stdout + res.stderr
    assert "passed" in res.stdout
