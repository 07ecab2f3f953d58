"""CPU: the oracle's C code under AddressSanitizer and
UndefinedBehaviorSanitizer.  tests/native/oracle_sanitize_driver.c calls every
exported oracle function on exactly sized heap buffers over degenerate and
ragged shapes; any out-of-bounds access or undefined behaviour aborts it."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_sanitized")
    cmd = ["gcc", "-O1", "-g", "-std=c11", "-fopenmp", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
           os.path.join(ROOT, "oracle", "oracle.c"), os.path.join(HERE, "native", "oracle_sanitize_driver.c"),
           "-o", exe]
    subprocess.check_call(cmd)
    env = dict(os.environ, OMP_NUM_THREADS="2", ASAN_OPTIONS="detect_leaks=1:abort_on_error=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "OK" in r.stdout
