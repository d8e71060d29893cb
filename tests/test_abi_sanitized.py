"""The HIP library's host code under AddressSanitizer and
UndefinedBehaviorSanitizer: a C driver calls the entry points that run on
the host alone (configuration validation, size queries, derived constants,
the argument checks of mclbm_create, the checkpoint-header parser on good
and damaged files).  The library is rebuilt for the test with the
sanitizers on its host code only (the device code is unchanged)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = "/opt/rocm/bin/hipcc"
CLANG = "/opt/rocm/llvm/bin/clang"

pytestmark = pytest.mark.slow


@pytest.mark.skipif(not (os.path.exists(HIPCC) and os.path.exists(CLANG)), reason="needs ROCm hipcc and clang")
def test_library_host_code_is_clean_under_sanitizers(tmp_path):
    lib = tmp_path / "libmclbm_asan.so"
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=undefined"]
    cmd = [HIPCC, "-O1", "-g", "-std=c++17", "-fPIC", "-shared", "--offload-arch=gfx950",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", *san,
           "-fno-omit-frame-pointer", "-I", os.path.join(ROOT, "include"), "-o", str(lib),
           os.path.join(ROOT, "paper_1511_04552_amd", "csrc", "mclbm.hip")]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    exe = tmp_path / "abi_driver"
    cmd = [CLANG, "-std=gnu11", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=undefined", "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(ROOT, "include"),
           os.path.join(ROOT, "tests", "sanitize", "abi_driver.c"), "-L", str(tmp_path), "-lmclbm_asan",
           "-L/opt/rocm/lib", "-lamdhip64", f"-Wl,-rpath,{tmp_path}", "-Wl,-rpath,/opt/rocm/lib", "-lm",
           "-o", str(exe)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1", UBSAN_OPTIONS="print_stacktrace=1")
    run = subprocess.run([str(exe), str(tmp_path)], capture_output=True, text=True, env=env, timeout=300)
    assert run.returncode == 0, run.stdout + run.stderr[-4000:]
    assert "abi host driver ok" in run.stdout
