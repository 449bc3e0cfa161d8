"""The oracle's pin tests under AddressSanitizer and UndefinedBehaviorSanitizer:
spgemm_oracle.c built with -fsanitize=address,undefined (every finding aborts)
and the whole pin suite run against that build in a child process."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _runtime(name):
    out = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True).stdout.strip()
    return out if os.path.isabs(out) and os.path.exists(out) else None


@pytest.mark.skipif(_runtime("libasan.so") is None, reason="gcc's AddressSanitizer runtime is not installed")
def test_pins_pass_under_asan_and_ubsan(tmp_path):
    sys.path.insert(0, ROOT)
    from oracle.build import build_oracle
    lib = build_oracle(force=True, sanitize=True, out=str(tmp_path / "liboracle_san.so"))
    env = dict(os.environ)
    env["ORACLE_LIB"] = lib
    env["LD_PRELOAD"] = _runtime("libasan.so")
    # Python itself is not instrumented: its allocations are not leaks of ours
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=1"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    env["OMP_NUM_THREADS"] = "4"
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_oracle_pins.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    tail = (r.stdout + r.stderr)[-3000:]
    assert r.returncode == 0, tail
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, tail
    assert " passed" in r.stdout, tail
