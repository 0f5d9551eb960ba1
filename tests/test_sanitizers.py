"""The oracle under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

Its pins (tests/test_oracle_pins.py) run again in a child process against a
sanitized build of oracle/dses_oracle.c; a report from either sanitizer aborts
that process and fails this test.  Device code has no such tool here; its
races would show up as determinism failures of the GPU tests (results come
from integer atomics and fixed-order reductions only).
"""
import os
import subprocess
import sys

import pytest

from oracle.build import build_oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _gcc_runtime(name):
    r = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True)
    path = r.stdout.strip()
    return path if os.path.isabs(path) and os.path.exists(path) else None


def test_oracle_pins_under_asan_and_ubsan(tmp_path):
    asan = _gcc_runtime("libasan.so")
    if asan is None:
        pytest.skip("gcc has no AddressSanitizer runtime")
    lib = build_oracle(out=str(tmp_path / "liboracle_asan_ubsan.so"), sanitize=True)
    env = dict(os.environ)
    # reports go to files: pytest's output capture would swallow them when a
    # sanitizer ends the child inside a test
    logs = tmp_path / "san"
    env.update(DSES_ORACLE_LIB=lib, LD_PRELOAD=asan,
               ASAN_OPTIONS=f"detect_leaks=0:halt_on_error=1:log_path={logs}",
               UBSAN_OPTIONS=f"halt_on_error=1:print_stacktrace=1:log_path={logs}")
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_oracle_pins.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    reports = "".join(f.read_text(errors="replace")[:4000]
                      for f in sorted(tmp_path.iterdir()) if f.name.startswith("san"))
    tail = r.stdout[-2000:] + "\n" + r.stderr[-2000:] + "\n" + reports
    assert r.returncode == 0 and not reports, tail
    assert " passed" in r.stdout, tail
