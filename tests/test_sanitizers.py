"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only, no GPU).

Builds tests/sanitize/driver.cpp with the library's host-side checks and exact Q reduction
(paper_2608_03695_amd/csrc/host.cpp) and the C oracle (oracle/mslm_oracle.c), all with
-fsanitize=address,undefined, and runs it: every validation path, the exact reduction on random
components of up to 64 slices, whole oracle solves (traced and not, 1 to 64 slices, weighted and
unit), and the oracle's big-integer comparator.  A sanitizer report or a failed check fails.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-fsanitize=address,undefined", "-fno-omit-frame-pointer", "-fno-sanitize-recover=all",
       "-g", "-O1"]


@pytest.mark.skipif(shutil.which("g++") is None or shutil.which("gcc") is None,
                    reason="needs gcc and g++")
def test_host_code_and_oracle_under_sanitizers(tmp_path):
    oracle_o = tmp_path / "oracle.o"
    subprocess.check_call(["gcc", *SAN, "-std=c11", "-c", os.path.join(ROOT, "oracle", "mslm_oracle.c"),
                           "-o", str(oracle_o)])
    exe = tmp_path / "driver"
    subprocess.check_call(["g++", *SAN, "-std=c++17",
                           os.path.join(ROOT, "tests", "sanitize", "driver.cpp"),
                           os.path.join(ROOT, "paper_2608_03695_amd", "csrc", "host.cpp"),
                           str(oracle_o), "-o", str(exe)])
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:halt_on_error=1:abort_on_error=0",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=600, env=env)
    assert out.returncode == 0, out.stderr[-4000:]
    assert "sanitized run ok" in out.stdout
