"""The oracle built with the address and undefined-behaviour sanitizers
(g++, host code only) and run over every entry point, dimension, boundary
type, order, splitting and limiter setting on small grids
(tests/oracle_sanitize_driver.cpp): no out-of-bounds access, use of freed
memory or undefined arithmetic.  CPU only."""
import os
import shutil
import subprocess
import tempfile

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


def test_oracle_under_address_and_ub_sanitizers():
    if shutil.which("g++") is None:
        pytest.skip("no g++")
    if os.environ.get("LD_PRELOAD"):
        pytest.skip("a preloaded library would come before the sanitizer runtime")
    with tempfile.TemporaryDirectory(prefix="tenoaa_san_") as tmp:
        exe = os.path.join(tmp, "oracle_san")
        cmd = ["g++", "-std=c++17", "-O1", "-g", "-ffp-contract=off", "-fno-omit-frame-pointer",
               "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
               os.path.join(HERE, "oracle_sanitize_driver.cpp"), "-o", exe]
        subprocess.run(cmd, check=True)
        env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
                   UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
        r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
        assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
        assert "0 failures" in r.stdout
        assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-4000:]
