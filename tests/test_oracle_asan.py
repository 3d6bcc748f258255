"""The C oracle built with AddressSanitizer and UndefinedBehaviorSanitizer
(gcc) and driven through every entry point on random tiny streams
(tests/oracle_asan_main.c): no memory error, leak or undefined behaviour."""
import os
import shutil
import subprocess
import tempfile

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_under_sanitizers():
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "oracle_asan")
        cmd = ["gcc", "-std=c11", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
               "-fno-sanitize-recover=undefined", os.path.join(ROOT, "oracle", "plds_oracle.c"),
               os.path.join(HERE, "oracle_asan_main.c"), "-o", exe, "-lm"]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0 and "asan" in (r.stderr or "").lower():
            pytest.skip("the AddressSanitizer runtime is not installed: " + r.stderr[-300:])
        assert r.returncode == 0, r.stderr
        env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:verify_asan_link_order=0", UBSAN_OPTIONS="print_stacktrace=1")
        r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
        assert r.returncode == 0, (r.stdout + r.stderr)[-4000:]
        assert "oracle driver ok" in r.stdout
        assert "runtime error" not in r.stderr, r.stderr[-4000:]
