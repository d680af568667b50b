"""The CPU oracle under AddressSanitizer and UndefinedBehaviorSanitizer: a C
driver (tests/sanitize_oracle_driver.c) runs every oracle entry point on
pseudo-random images of odd sizes; any out-of-bounds access, use after free,
leak, signed overflow or other undefined behaviour aborts it."""
import os
import shutil
import subprocess

import pytest

import oracle

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
@pytest.mark.parametrize("openmp", [False, True], ids=["serial", "openmp"])
def test_oracle_is_clean_under_sanitizers(tmp_path, openmp):
    exe = tmp_path / "driver"
    cmd = ["gcc", "-O1", "-g", "-std=gnu99", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-Wno-unknown-pragmas", *(["-fopenmp"] if openmp else []),
           "-o", str(exe), os.path.join(HERE, "sanitize_oracle_driver.c"), oracle.SRC]
    subprocess.run(cmd, check=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1", OMP_NUM_THREADS="4")
    r = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    assert "sanitized oracle runs" in r.stdout
