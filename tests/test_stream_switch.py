"""Host check of the context's stream hand-off (csrc/ram_stream.h): calls of one
context issued on different streams must run one after the other on its shared
scratch.  Built with g++ (no GPU, no HIP headers) and run against a stand-in
runtime that tracks what each stream's next work is ordered after."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2305_05362_amd", "csrc")
SRC = os.path.join(ROOT, "tests", "host", "stream_switch_check.cpp")


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_stream_handoff(tmp_path):
    exe = str(tmp_path / "stream_switch_check")
    subprocess.run(["g++", "-std=c++17", "-O1", "-Wall", "-Werror", "-g",
                    "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                    "-I", CSRC, SRC, "-o", exe], check=True)
    out = subprocess.run([exe], capture_output=True, text=True)
    assert out.returncode == 0, out.stdout + out.stderr
    assert "all checks passed" in out.stdout
