"""The C ABI's host code under AddressSanitizer and UndefinedBehaviorSanitizer
(CPU): parameter derivation, workspace layout, argument checks of create and
of the allocation-free entry point, and the autotune cache file.  The
library's host sources are compiled with the sanitizers (its kernels without),
linked into tests/capi_host_driver.cpp, and run without a GPU."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_1401_0188_amd", "csrc")
HIPCC = "/opt/rocm/bin/hipcc"
CLANG = "/opt/rocm/lib/llvm/bin/clang++"
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all"]


@pytest.mark.skipif(not (os.path.exists(HIPCC) and os.path.exists(CLANG)), reason="ROCm compilers not available")
def test_capi_host_code_is_clean_under_sanitizers(tmp_path):
    t = str(tmp_path)
    host_san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                "-Xarch_host", "-fno-sanitize-recover=all"]
    base = [HIPCC, "--offload-arch=gfx950", "-std=c++17", "-O1", "-g", "-I" + os.path.join(ROOT, "include")]
    subprocess.check_call(base + ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-fPIC", "-x", "hip",
                                  "-c", os.path.join(CSRC, "lbm13_kernels.hip"), "-o", t + "/k.o"])
    subprocess.check_call(base + host_san + ["-c", os.path.join(CSRC, "lbm13_capi.cpp"), "-o", t + "/c.o"])
    subprocess.check_call([CLANG, "-std=c++17", "-O1", "-g"] + SAN +
                          ["-c", os.path.join(CSRC, "lbm13_tune_cache.cpp"), "-o", t + "/t.o"])
    subprocess.check_call([CLANG, "-std=c++17", "-O1", "-g"] + SAN +
                          ["-c", os.path.join(HERE, "capi_host_driver.cpp"), "-o", t + "/d.o"])
    subprocess.check_call(base + host_san[:4] + [t + "/k.o", t + "/c.o", t + "/t.o", t + "/d.o", "-o", t + "/drv"])
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1",
               HIP_VISIBLE_DEVICES="")
    r = subprocess.run([t + "/drv"], capture_output=True, text=True, timeout=300, env=env, cwd=t)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "0 failure(s)" in r.stdout
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr
