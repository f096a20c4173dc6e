"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (no GPU).

* The FP64 oracle (oracle/ram_oracle.c) built with -fsanitize=address,undefined
  runs the oracle pin tests (tests/test_oracle_*.py) in a child process.
* The C ABI's host layer (csrc/ram_api.cpp: argument checks, layout checks,
  error reporting) built the same way with g++, linked with the library's
  HIP objects as built (their host halves are launch wrappers; the device
  code is not instrumented), runs tests/test_abi.py's error paths.

Any sanitizer report ends the child with a nonzero status (halt on the first
error).  Leak detection is off: the Python interpreter itself keeps memory
until exit.
"""
import glob
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2305_05362_amd", "csrc")
BUILD = os.path.join(ROOT, "paper_2305_05362_amd", "_build")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]


def _runtime():
    if shutil.which("gcc") is None:
        return None
    p = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True,
                       text=True).stdout.strip()
    return p if os.path.isabs(p) and os.path.exists(p) else None


ASAN = _runtime()
needs_asan = pytest.mark.skipif(ASAN is None, reason="needs gcc's ASan runtime")


def _env(**extra):
    env = dict(os.environ)
    env["LD_PRELOAD"] = ASAN
    env["ASAN_OPTIONS"] = "detect_leaks=0:halt_on_error=1:abort_on_error=0"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    env["OMP_NUM_THREADS"] = "4"
    env.update(extra)
    return env


def _run(args, env, cwd):
    out = subprocess.run(args, env=env, cwd=cwd, capture_output=True, text=True,
                         timeout=600)
    text = out.stdout[-4000:] + out.stderr[-4000:]
    assert out.returncode == 0, text
    assert "ERROR: AddressSanitizer" not in text, text
    assert "runtime error:" not in text, text
    return text


@needs_asan
def test_oracle_pins_under_asan_ubsan(tmp_path):
    lib = str(tmp_path / "libram_oracle_san.so")
    subprocess.run(["gcc", "-O1", "-g", *SAN, "-ffp-contract=off", "-fopenmp", "-fPIC",
                    "-shared", "-std=c11", "-Wall", "-o", lib,
                    os.path.join(ROOT, "oracle", "ram_oracle.c"), "-lm"], check=True)
    tests = sorted(glob.glob(os.path.join(ROOT, "tests", "test_oracle_*.py")))
    assert tests
    text = _run([sys.executable, "-m", "pytest", "-q", "-x", "-m", "not gpu",
                 "-p", "no:cacheprovider", *tests], _env(RAM_ORACLE_LIB=lib), ROOT)
    assert " passed" in text


@needs_asan
@pytest.mark.skipif(shutil.which("g++") is None or not os.path.isdir("/opt/rocm/include"),
                    reason="needs g++ and the ROCm headers")
def test_abi_error_paths_under_asan_ubsan(tmp_path):
    objs = sorted(glob.glob(os.path.join(BUILD, "*.o")))
    objs = [o for o in objs if os.path.basename(o) != "ram_api.o"]
    if not objs:
        pytest.skip("the library's HIP objects are not built (python -m paper_2305_05362_amd.build)")
    api = str(tmp_path / "ram_api_san.o")
    lib = str(tmp_path / "libram_san.so")
    subprocess.run(["g++", "-std=c++17", "-O1", "-g", *SAN, "-fPIC", "-D__HIP_PLATFORM_AMD__",
                    "-I", "/opt/rocm/include", "-I", os.path.join(ROOT, "include"),
                    "-I", CSRC, "-c", os.path.join(CSRC, "ram_api.cpp"), "-o", api],
                   check=True)
    subprocess.run(["g++", "-shared", *SAN, "-o", lib, api, *objs, "-L/opt/rocm/lib",
                    "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib"], check=True)
    driver = ("import sys, pytest\n"
              "from paper_2305_05362_amd import _lib\n"
              f"_lib.load_library({lib!r})\n"
              "sys.exit(pytest.main(['-q', '-x', '-p', 'no:cacheprovider', "
              f"{os.path.join(ROOT, 'tests', 'test_abi.py')!r}]))\n")
    text = _run([sys.executable, "-c", driver], _env(), ROOT)
    assert " passed" in text
