"""The C oracle built with the address and undefined-behaviour sanitizers (gcc, host code
only) runs every entry point on small seeded problems without a report."""
import os
import shutil
import subprocess
import tempfile

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ORACLE = os.path.join(os.path.dirname(HERE), "oracle")


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_oracle_under_sanitizers():
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "drv")
        cmd = ["gcc", "-O1", "-g", "-std=c99", "-fopenmp", "-fno-omit-frame-pointer",
               "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-I", ORACLE,
               os.path.join(ORACLE, "sdlref.c"), os.path.join(HERE, "oracle_sanitize_driver.c"), "-o", exe, "-lm"]
        subprocess.run(cmd, check=True, capture_output=True, text=True)
        env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0", OMP_NUM_THREADS="2")
        res = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
        assert res.returncode == 0, res.stdout + res.stderr
        assert "ok" in res.stdout
        assert "runtime error" not in res.stderr and "AddressSanitizer" not in res.stderr, res.stderr
