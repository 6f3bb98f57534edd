"""The library's host code under AddressSanitizer and UndefinedBehavior-
Sanitizer (no GPU): every HIP source is compiled with the sanitizers on its
host side only (device code is built as usual), linked with
tests/host_abi_check.cpp, which drives the C ABI through every path that
runs before a launch -- argument and option checks, workspace sizing, the
no-allocation entry point's size check, the batched option checks, model
blob validation -- and must exit cleanly."""
import concurrent.futures as cf
import glob
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "bin", "hipcc")
FLAGS = ["--offload-arch=gfx950", "-O1", "-g", "-std=c++17",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
         "-Xarch_host", "-fno-omit-frame-pointer", "-I", os.path.join(ROOT, "include")]


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not installed")
def test_host_abi_paths_clean_under_asan_and_ubsan(tmp_path):
    srcs = sorted(glob.glob(os.path.join(ROOT, "paper_2302_12199_amd", "csrc", "*.hip")))
    srcs.append(os.path.join(ROOT, "tests", "host_abi_check.cpp"))

    def compile_one(src):
        obj = str(tmp_path / (os.path.basename(src) + ".o"))
        r = subprocess.run([HIPCC, *FLAGS, "-c", src, "-o", obj], capture_output=True,
                           text=True)
        return obj, r

    with cf.ThreadPoolExecutor(min(8, os.cpu_count() or 1)) as ex:
        results = list(ex.map(compile_one, srcs))
    for obj, r in results:
        assert r.returncode == 0, r.stderr[-2000:]
    exe = str(tmp_path / "host_abi_check")
    r = subprocess.run([HIPCC, *FLAGS, *[o for o, _ in results], "-o", exe],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, (r.stdout + r.stderr)[-4000:]
    assert "host ABI checks passed" in r.stdout
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr
