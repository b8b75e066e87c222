"""The CPU oracle under AddressSanitizer and UndefinedBehaviorSanitizer.

tests/sanitize/oracle_driver.c calls every oracle entry point (runs, extended
runs, powers, Algorithm 1 and 2 trees, the sort with every option, the batched
sort) on seeded inputs of 0..20011 keys with ties, for all key types and
k in {2, 3, 4, 8}.  The build stops at the first sanitizer report, so a clean
exit means no out-of-bounds access, leak or undefined arithmetic on those
inputs.  CPU only; skipped where gcc has no sanitizer runtime.
"""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_oracle_clean_under_asan_ubsan(tmp_path):
    exe = str(tmp_path / "oracle_asan")
    cmd = ["gcc", "-std=c11", "-g", "-O1", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
           "-I", os.path.join(ROOT, "oracle"),
           os.path.join(ROOT, "oracle", "oracle.c"),
           os.path.join(ROOT, "tests", "sanitize", "oracle_driver.c"), "-o", exe]
    b = subprocess.run(cmd, capture_output=True, text=True)
    if b.returncode != 0 and ("asan" in b.stderr.lower() or "ubsan" in b.stderr.lower()):
        pytest.skip("no sanitizer runtime for gcc here: " + b.stderr[-300:])
    assert b.returncode == 0, b.stderr
    # a library preloaded by the environment would come before the sanitizer
    # runtime; tell it not to insist on being first
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, (r.stdout + r.stderr)[-4000:]
    assert "all cases passed" in r.stdout
