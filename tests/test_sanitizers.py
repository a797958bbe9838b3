"""AddressSanitizer + UndefinedBehaviorSanitizer runs of the CPU-side code:
the oracle's C (built with gcc) and the library's host code (the C ABI's
validation, tuning-table parser, rules and plans; compiled with the host
half instrumented and linked with the library's other objects).  The
drivers in tests/sanitize/ only make calls that return before any device
work, so both run on a machine without a GPU."""
import glob
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests", "sanitize")
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")


def test_oracle_under_asan_and_ubsan(tmp_path):
    exe = str(tmp_path / "oracle_asan")
    subprocess.run(["gcc", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
                    "-fno-omit-frame-pointer", "-g", "-O1", "-fopenmp",
                    os.path.join(ROOT, "oracle", "oracle.c"), os.path.join(HERE, "oracle_driver.c"),
                    "-o", exe, "-lm"], check=True)
    r = subprocess.run([exe], env=ENV, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-4000:]


def test_host_abi_under_asan_and_ubsan(tmp_path):
    from paper_2305_18236_amd import build as libbuild
    objs = [o for o in glob.glob(os.path.join(libbuild.BUILD, "*.o")) if not o.endswith("mgemm_api.o")]
    if not objs or shutil.which(libbuild.hipcc()) is None and not os.path.exists(libbuild.hipcc()):
        pytest.skip("library objects not built")
    clangxx = os.path.join(os.path.dirname(libbuild.hipcc()), "..", "llvm", "bin", "clang++")
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer", "-g"]
    api = str(tmp_path / "mgemm_api_san.o")
    drv = str(tmp_path / "abi_driver.o")
    exe = str(tmp_path / "abi_asan")
    flags = [f for f in libbuild.DEVICE_FLAGS if f != "-Wall"]
    subprocess.run([libbuild.hipcc(), *flags, *san, "-c", os.path.join(libbuild.CSRC, "mgemm_api.hip"), "-o", api],
                   check=True)
    subprocess.run([clangxx, "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-c",
                    os.path.join(HERE, "abi_driver.cpp"), "-o", drv], check=True)
    rocm = os.path.dirname(os.path.dirname(libbuild.hipcc()))
    subprocess.run([clangxx, "-fsanitize=address,undefined", drv, api, *objs, "-o", exe,
                    "-L" + os.path.join(rocm, "lib"), "-lamdhip64", "-Wl,-rpath," + os.path.join(rocm, "lib")],
                   check=True)
    r = subprocess.run([exe], env=ENV, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-4000:]
