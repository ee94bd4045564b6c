"""The oracle under AddressSanitizer, LeakSanitizer and
UndefinedBehaviorSanitizer: tests/oracle_sanitize_main.c drives it through
every kernel family, calibrated and given r1, r2, the three DataReduct
methods, the swap pass, duplicate points and a single point; any invalid
access, leak or undefined operation aborts the run (CPU only)."""
import os
import shutil
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_oracle_clean_under_sanitizers():
    if shutil.which("gcc") is None:
        pytest.skip("no gcc")
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "h2o_san")
        cmd = ["gcc", "-O1", "-g", "-std=c11", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
               "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer",
               "-o", exe, os.path.join(ROOT, "oracle", "h2o.c"),
               os.path.join(ROOT, "tests", "oracle_sanitize_main.c"), "-lm"]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0 and "sanitize" in r.stderr:
            pytest.skip("gcc without sanitizer runtimes")
        assert r.returncode == 0, r.stderr[-2000:]
        env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1", OMP_NUM_THREADS="2")
        r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
        assert r.returncode == 0, (r.stdout + r.stderr)[-4000:]
        assert r.stdout.count(" ok\n") == 8, r.stdout
