"""The oracle's pins again, against its AddressSanitizer + UndefinedBehaviorSanitizer build.

The oracle is plain C run on host memory that Python hands it; an out-of-bounds index, a use of
freed memory or undefined arithmetic in it would not show in the ordinary pins.  This runs the
oracle's CPU pins in a child interpreter that loads ``liboracle_san.so`` (any report aborts it)
with the ASan runtime preloaded, and requires a clean exit.
"""
from __future__ import annotations

import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _libasan() -> str:
    p = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True, check=True)
    return p.stdout.strip()


def test_oracle_pins_clean_under_asan_and_ubsan():
    from oracle.make_lib import build

    build(sanitize=True)
    asan = _libasan()
    if not os.path.isabs(asan) or not os.path.exists(asan):
        pytest.skip("gcc has no AddressSanitizer runtime here")
    env = dict(os.environ)
    env["LDO_SANITIZE"] = "1"
    env["LD_PRELOAD"] = asan + (":" + env["LD_PRELOAD"] if env.get("LD_PRELOAD") else "")
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=1"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1"
    env["PYTHONPATH"] = ROOT + (os.pathsep + env["PYTHONPATH"] if env.get("PYTHONPATH") else "")
    cmd = [sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider", "-m", "not gpu",
           os.path.join(ROOT, "tests", "test_oracle_pins.py"), os.path.join(ROOT, "tests", "test_oracle_trees.py"),
           os.path.join(ROOT, "tests", "test_oracle_taylor.py"), os.path.join(ROOT, "tests", "test_oracle_lanczos.py"),
           "-k", "not statistical and not grid32_closed_form"]
    p = subprocess.run(cmd, cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    out = p.stdout + p.stderr
    assert "AddressSanitizer" not in out and "runtime error" not in out, out[-4000:]
    assert p.returncode == 0, out[-4000:]
    assert " passed" in out
