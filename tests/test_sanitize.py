"""The CPU oracle and the event generator built with AddressSanitizer and
UndefinedBehaviorSanitizer (gcc), run on small inputs of every scene and
flag combination (``tests/sanitize_driver.c``).  Any out-of-bounds access,
use after free, leak, signed overflow or other undefined behaviour aborts the
run with the sanitizer's report."""
from __future__ import annotations

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

pytestmark = pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not found")


def test_oracle_and_generator_under_sanitizers(tmp_path):
    exe = str(tmp_path / "sanitize_driver")
    cmd = ["gcc", "-std=gnu99", "-O1", "-g", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-static-libasan", "-static-libubsan", "-pthread", "-Wall",
           "-o", exe, os.path.join(ROOT, "tests", "sanitize_driver.c"),
           os.path.join(ROOT, "oracle", "esi_oracle.c"), "-lm"]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    env = dict(os.environ)
    env["ASAN_OPTIONS"] = "detect_leaks=1:abort_on_error=0:halt_on_error=1"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-4000:])
    assert r.stdout.strip().endswith("ok")
    assert "runtime error" not in r.stderr and "Sanitizer" not in r.stderr, r.stderr[-4000:]
