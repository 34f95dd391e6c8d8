"""The library's host code under the sanitizers: host_spgemm.cpp (the
multithreaded CPU hash SpGEMM) built with AddressSanitizer +
UndefinedBehaviorSanitizer and, separately, ThreadSanitizer, driven by
tests/sanitize/host_spgemm_check.cpp (random products on 1 and 4 threads,
bit-exact against an ordered-map accumulation; structure checks).  Host
compiler only, no GPU."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2002_10083_amd", "csrc")
DRIVER = os.path.join(ROOT, "tests", "sanitize", "host_spgemm_check.cpp")

pytestmark = pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")


@pytest.mark.parametrize("kind,flags", [
    ("asan_ubsan", ["-fsanitize=address,undefined", "-fno-sanitize-recover=all"]),
    ("tsan", ["-fsanitize=thread"]),
])
def test_host_spgemm_under_sanitizer(tmp_path, kind, flags):
    exe = str(tmp_path / ("check_" + kind))
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-ffp-contract=off", "-pthread",
           *flags, "-I" + CSRC, DRIVER, os.path.join(CSRC, "host_spgemm.cpp"), "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0 and "cannot find" in (r.stderr or ""):
        pytest.skip("sanitizer runtime not installed: " + r.stderr.strip().splitlines()[-1])
    assert r.returncode == 0, r.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", TSAN_OPTIONS="halt_on_error=1")
    p = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert p.returncode == 0, p.stdout + p.stderr
    assert p.stdout.strip() == "ok"
    assert "runtime error" not in p.stderr and "Sanitizer" not in p.stderr, p.stderr
