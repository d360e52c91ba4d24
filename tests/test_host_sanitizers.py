"""The library's host code (parameter derivation, validation, workspace
layout) built with AddressSanitizer and UndefinedBehaviorSanitizer, and run
on a fuzzed stream of valid and invalid parameter sets (tests/host/derive_fuzz.c).
Only host code is instrumented: every -fsanitize option of the hipcc lines is
given to the host pass alone. Needs no GPU (no device call is made)."""
import concurrent.futures
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2101_07088_amd", "csrc")
SOURCES = ["plan.cpp", "k_particles.hip", "k_grid.hip", "k_fft.hip", "k_column.hip"]
HOST_SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer"]


def _tool(name):
    for cand in (os.path.join("/opt/rocm/bin", name), os.path.join("/opt/rocm/llvm/bin", name), shutil.which(name)):
        if cand and os.path.exists(cand):
            return cand
    return None


def test_host_code_under_asan_and_ubsan(tmp_path):
    hipcc, clangxx = _tool("hipcc"), _tool("clang++")
    if not hipcc or not clangxx:
        pytest.skip("hipcc / clang++ not available")
    inc = ["-I", os.path.join(ROOT, "include"), "-I", CSRC]
    arch = os.environ.get("DPSE_OFFLOAD_ARCH", "gfx950")

    def compile_one(src):
        obj = str(tmp_path / (os.path.splitext(src)[0] + ".o"))
        cmd = [hipcc, "-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj, f"--offload-arch={arch}", "-O1", "-g",
               "-std=c++17", "-fPIC", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"] + HOST_SAN + inc
        r = subprocess.run(cmd, capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-3000:]
        return obj

    with concurrent.futures.ThreadPoolExecutor(max_workers=5) as ex:
        objs = list(ex.map(compile_one, SOURCES))
    drv = str(tmp_path / "derive_fuzz.o")
    r = subprocess.run([clangxx, "-x", "c", "-c", os.path.join(ROOT, "tests", "host", "derive_fuzz.c"), "-o", drv,
                        "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined"] + inc,
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    exe = str(tmp_path / "derive_fuzz")
    r = subprocess.run([clangxx, "-fsanitize=address,undefined", drv] + objs +
                       ["-L/opt/rocm/lib", "-Wl,-rpath,/opt/rocm/lib", "-lamdhip64", "-o", exe],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe, "8000"], capture_output=True, text=True, env=env, timeout=600)
    print(r.stdout, r.stderr[-2000:])
    assert r.returncode == 0, r.stdout + r.stderr[-4000:]
    assert "0 failed checks" in r.stdout
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr
