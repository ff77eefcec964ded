"""The oracle's C code under AddressSanitizer and UndefinedBehaviorSanitizer:
an instrumented build runs the oracle pins in a child process (CPU only).
Any out-of-bounds access, use after free or undefined behaviour aborts the
child and fails this test."""

import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _runtime(name):
    try:
        path = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True,
                              check=True).stdout.strip()
    except (OSError, subprocess.CalledProcessError):
        return None
    return path if os.path.isabs(path) and os.path.exists(path) else None


@pytest.mark.skipif(_runtime("libasan.so") is None, reason="gcc's ASan runtime is not installed")
def test_oracle_pins_under_sanitizers(tmp_path):
    sys.path.insert(0, ROOT)
    from oracle import build as ob

    lib = ob.build_sanitized(str(tmp_path / "liboracle_asan.so"))
    env = dict(os.environ)
    env.update({
        "DI_ORACLE_LIB": lib,
        "LD_PRELOAD": _runtime("libasan.so"),
        # the interpreter itself is not instrumented: no leak report at exit
        "ASAN_OPTIONS": "detect_leaks=0:abort_on_error=1",
        "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1",
        "PYTHONPATH": ROOT,
    })
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_oracle_pins.py"),
                        os.path.join(ROOT, "tests", "test_dataset2_like.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-3000:]
    assert "passed" in r.stdout
