"""The C oracle under AddressSanitizer and UndefinedBehaviorSanitizer.

tests/sanitize_driver.c runs the oracle end to end on a small seeded input
(statistics, projections, r, hashing, packing, the LSH search under every
stopping rule with and without its trace and fallback, both exact top-k
routines); here it is built with gcc and both sanitizers, every finding
fatal, and must exit cleanly and print "ok".
"""
import os
import shutil
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRCS = [os.path.join(ROOT, "oracle", "momenti_oracle.c"), os.path.join(ROOT, "oracle", "o1fast.c"),
        os.path.join(ROOT, "tests", "sanitize_driver.c")]


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not found")
def test_oracle_is_clean_under_asan_and_ubsan():
    with tempfile.TemporaryDirectory() as tmp:
        exe = os.path.join(tmp, "orc_san")
        cmd = ["gcc", "-O1", "-g", "-std=c11", "-D_GNU_SOURCE", "-ffp-contract=off", "-fno-omit-frame-pointer",
               "-fsanitize=address,undefined", "-fno-sanitize-recover=all", *SRCS, "-lm", "-o", exe]
        subprocess.run(cmd, check=True, capture_output=True, text=True)
        env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
                   UBSAN_OPTIONS="print_stacktrace=1")
        r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
        assert r.returncode == 0, r.stderr[-4000:]
        assert r.stdout.strip() == "ok", (r.stdout, r.stderr[-2000:])
