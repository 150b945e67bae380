"""The oracle under AddressSanitizer and UndefinedBehaviorSanitizer (host code,
CPU only): a C++ driver calls every entry point on small, edge-case and
invalid inputs; any sanitizer report fails the test."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ is not installed")
def test_oracle_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_sanitize")
    cmd = ["g++", "-O1", "-g", "-std=c++17", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           os.path.join(HERE, "oracle_sanitize.cpp"), os.path.join(ROOT, "oracle", "wrs_oracle.cpp"),
           os.path.join(ROOT, "oracle", "wrs_oracle_os.cpp"), "-o", exe]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    # the environment is kept as it is (a preloaded library may precede the
    # sanitizer runtime, so its link-order check is off)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, r.stderr[-3000:]
    assert "oracle sanitize" in r.stdout
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-3000:]
