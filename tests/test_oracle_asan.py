"""The CPU oracle under host AddressSanitizer and UndefinedBehaviorSanitizer.

oracle/oracle.c is compiled with tests/asan_oracle_main.c into one executable
with gcc -fsanitize=address,undefined (no recovery) and run: every routine on
small operators with projector blocks, a ragged grid, one plane, nf = 1 and no
projectors.  Any out-of-bounds access, leak or undefined operation fails it."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_oracle_clean_under_address_and_ub_sanitizers(tmp_path):
    exe = tmp_path / "oracle_asan"
    cmd = ["gcc", "-std=c11", "-g", "-O1", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           os.path.join(HERE, "asan_oracle_main.c"), "-o", str(exe), "-lm"]
    subprocess.run(cmd, check=True, cwd=ROOT)
    # verify_asan_link_order=0: the environment may preload other libraries
    env = dict(os.environ,
               ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stderr[-4000:]
    assert "oracle sanitizer run ok" in r.stdout
