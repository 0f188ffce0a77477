"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer: the
oracle's C part (tree builds, Barnes-Hut forces and energies, direct sums) and
the C ABI's host paths (argument validation of the entry points, the host
Kabsch solver), each driven by a small program in tests/sanitize/. CPU only:
the device code is built without sanitizers and never launched."""
import concurrent.futures as cf
import glob
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = os.path.join(ROOT, "tests", "sanitize")
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
           UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")


def _run(exe):
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=ENV)
    assert r.returncode == 0, (r.stdout + r.stderr)[-4000:]
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-4000:]
    return r.stdout


def test_oracle_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_driver")
    subprocess.check_call(["gcc", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                           "-fno-sanitize-recover=all", "-fopenmp",
                           os.path.join(ROOT, "oracle", "fga_oracle.c"),
                           os.path.join(SAN, "oracle_driver.c"), "-o", exe, "-lm"])
    assert "oracle driver ok" in _run(exe)


@pytest.mark.skipif(not os.path.exists("/opt/rocm/bin/hipcc"), reason="needs hipcc")
def test_abi_host_paths_under_sanitizers(tmp_path):
    hipcc = "/opt/rocm/bin/hipcc"
    inc = ["-I", os.path.join(ROOT, "include"), "-I", os.path.join(ROOT, "paper_2009_14005_amd", "csrc")]
    host_san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer"]

    def compile_one(src):
        obj = str(tmp_path / (os.path.basename(src) + ".o"))
        subprocess.run([hipcc, "--offload-arch=gfx950", "-O1", "-g", "-fPIC", "-std=c++17",
                        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"] + host_san + inc +
                       ["-c", src, "-o", obj], check=True, capture_output=True)
        return obj
    srcs = sorted(glob.glob(os.path.join(ROOT, "paper_2009_14005_amd", "csrc", "*.hip")))
    with cf.ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        objs = list(ex.map(compile_one, srcs))
    drv = str(tmp_path / "abi_driver.o")
    subprocess.run([hipcc, "-O1", "-g", "-std=c++17"] + host_san + inc +
                   ["-c", os.path.join(SAN, "abi_driver.cpp"), "-o", drv], check=True, capture_output=True)
    exe = str(tmp_path / "abi_driver")
    subprocess.run([hipcc, "--offload-arch=gfx950", "-fsanitize=address,undefined", "-fno-gpu-sanitize"] +
                   objs + [drv, "-o", exe], check=True, capture_output=True)
    assert "abi driver ok" in _run(exe)
