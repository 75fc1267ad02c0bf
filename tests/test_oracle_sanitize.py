"""The CPU oracle under AddressSanitizer, LeakSanitizer and UndefinedBehaviorSanitizer.

tests/oracle_sanitize_driver.c compiles oracle/lbpf_ref.c into one program with
the sanitizers and runs every exported routine on seeded inputs that reach the
edges (3 x 3 crops, crops on every border, all-zero depth, the 256-bin mapping,
single-channel modalities, warped crops at the plane's last row and column,
rejected arguments, training and tracking). Any out-of-bounds access, leak or
undefined operation aborts the program. Host code only: nothing here touches
the GPU library.
"""
import os
import shutil
import subprocess
from pathlib import Path

import pytest

ROOT = Path(__file__).resolve().parent.parent


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_oracle_clean_under_sanitizers(tmp_path):
    exe = tmp_path / "oracle_sanitize"
    build = ["gcc", "-std=c11", "-O1", "-g", "-fsanitize=address,undefined",
             "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-Wall", "-Wextra",
             "-I", str(ROOT / "oracle"), str(ROOT / "tests" / "oracle_sanitize_driver.c"),
             "-o", str(exe), "-lpthread", "-lm"]
    r = subprocess.run(build, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "oracle sanitize ok" in r.stdout
    assert "runtime error" not in r.stderr and "Sanitizer" not in r.stderr, r.stderr
