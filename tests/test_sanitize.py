"""The host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU):
the symbolic analysis (every ordering and relaxation, groups, malformed
patterns) and the C oracle (factor, solves, scaling, refinement, the 4x4
system) driven on seeded random inputs by tests/sanitize/host_driver.cpp,
built with g++/gcc and -fsanitize=address,undefined. Any sanitizer report
ends the driver with a non-zero status."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
pytestmark = pytest.mark.slow


def test_host_code_under_sanitizers(tmp_path):
    if not shutil.which("g++") or not shutil.which("gcc"):
        pytest.skip("no host compiler")
    san = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g", "-O1"]
    orc_o = str(tmp_path / "oracle.o")
    subprocess.check_call(["gcc", "-std=c11", "-ffp-contract=off", *san, "-c", "-o", orc_o,
                           os.path.join(ROOT, "oracle", "oracle.c")])
    exe = str(tmp_path / "host_driver")
    subprocess.check_call(["g++", "-std=c++17", *san, "-o", exe,
                           os.path.join(ROOT, "tests", "sanitize", "host_driver.cpp"),
                           os.path.join(ROOT, "paper_2110_03636_amd", "csrc", "analysis.cpp"), orc_o, "-lm"])
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    res = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    assert res.returncode == 0, res.stdout[-4000:] + res.stderr[-8000:]
    assert "0 failed checks" in res.stdout
