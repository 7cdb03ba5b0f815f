"""The CPU oracle built with AddressSanitizer and UndefinedBehaviorSanitizer
(g++ -fsanitize=address,undefined, errors fatal) runs every entry point on
small seeded clouds through tests/oracle_sanitize_main.cpp.  CPU only."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_oracle_under_address_and_ub_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_sanitized")
    subprocess.check_call([
        "g++", "-O1", "-g", "-std=c++17", "-fsanitize=address,undefined",
        "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
        os.path.join(ROOT, "oracle", "ph0_oracle.cpp"),
        os.path.join(ROOT, "tests", "oracle_sanitize_main.cpp"), "-o", exe])
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "cases ok" in r.stdout
