"""Host-side defect validation, quantisation and footprint enumeration of the
library source, built for the host with AddressSanitizer and
UndefinedBehaviorSanitizer (tests/host/host_checks.cpp) and run on the CPU:
every footprint equals a brute-force membership scan of the grid, invalid
records are refused with a message, and the sanitizers report nothing."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


@pytest.mark.skipif(not os.path.exists(HIPCC) and not shutil.which("hipcc"), reason="hipcc not installed")
def test_host_code_under_asan_and_ubsan(tmp_path):
    exe = str(tmp_path / "host_checks")
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer"]
    cmd = [
        HIPCC, "-O1", "-g", "-std=c++17", "--offload-arch=gfx950",
        f"-I{os.path.join(ROOT, 'include')}", f"-I{os.path.join(ROOT, 'paper_2403_09158_amd', 'csrc')}",
        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-Wno-unused-command-line-argument",
        *san, os.path.join(HERE, "host", "host_checks.cpp"), "-o", exe,
        "-fsanitize=address,undefined", "-Wl,--unresolved-symbols=ignore-all",
    ]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-4000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=600, env=env)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-4000:])
    assert "ok: 0 failure(s)" in r.stdout
