"""The host side of the C ABI under AddressSanitizer and UndefinedBehavior-
Sanitizer: tests/host/abi_host_checks.cpp (validation and error paths, host
coarsening, footprint, null handles) is built together with the library
sources, the sanitizers on host code only, and must run clean. CPU only."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = "/opt/rocm/bin/hipcc"


def test_abi_host_paths_run_clean_under_sanitizers(tmp_path):
    if not os.path.exists(HIPCC) or shutil.which("gcc") is None:
        pytest.skip("hipcc not available")
    exe = tmp_path / "abi_host_checks"
    # sanitizers on the host pass only (each flag after -Xarch_host); the
    # device code is built as in the library
    sanitize = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                "-Xarch_host", "-fno-sanitize-recover=undefined"]
    cmd = ([HIPCC, "--offload-arch=gfx950", "-std=c++17", "-O1", "-g", "-Xclang", "-target-feature", "-Xclang",
            "-packed-fp32-ops"] + sanitize +
           ["-I", os.path.join(ROOT, "include"), os.path.join(ROOT, "tests", "host", "abi_host_checks.cpp"),
            os.path.join(ROOT, "paper_2505_05424_amd", "csrc", "dotsocp.hip"), "-o", str(exe)])
    subprocess.run(cmd, check=True, capture_output=True, timeout=600)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300, env=env)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "OK (0 failures)" in r.stdout
