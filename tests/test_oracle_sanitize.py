"""The C oracle built with AddressSanitizer and UndefinedBehaviorSanitizer (a
plain gcc build of oracle/bfs_oracle.c with tests/oracle_sanitize.c, no GPU
code) runs every entry point on awkward small graphs without a report."""
import os
import shutil
import subprocess
import tempfile

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_clean_under_asan_ubsan():
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "oracle_sanitize")
        cmd = ["gcc", "-std=c11", "-D_POSIX_C_SOURCE=199309L", "-O1", "-g", "-fno-omit-frame-pointer",
               "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
               "-o", exe, os.path.join(ROOT, "oracle", "bfs_oracle.c"), os.path.join(HERE, "oracle_sanitize.c")]
        subprocess.run(cmd, check=True, capture_output=True, text=True)
        # verify_asan_link_order=0: the environment may preload a library of
        # its own ahead of the sanitizer runtime; that is not a finding
        env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:verify_asan_link_order=0",
                   UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
        r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=120)
        assert r.returncode == 0, r.stdout + r.stderr
        assert "0 failures" in r.stdout
