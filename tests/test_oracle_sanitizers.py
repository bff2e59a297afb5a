"""The CPU oracle under AddressSanitizer and UndefinedBehaviorSanitizer.

A small C driver (tests/sanitize/oracle_driver.c) runs every process of the
oracle, with two species, an E grid, a magnetic map, self-consistent
electrons, the heating kick and (second pass) the tracked-neutral
density and exchange partners, sorts every 7 steps and round-trips the
state; the build aborts on the first invalid access, leak or undefined
operation.  Host code only, built with gcc.
"""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_oracle_runs_clean_under_asan_and_ubsan(tmp_path):
    exe = str(tmp_path / "oracle_driver")
    cmd = ["gcc", "-O1", "-g", "-std=c11", "-ffp-contract=off", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
           "-I", os.path.join(ROOT, "oracle"), os.path.join(HERE, "sanitize", "oracle_driver.c"),
           os.path.join(ROOT, "oracle", "ecr_oracle.c"), "-lm", "-o", exe]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stderr[-4000:]
    assert "ERROR" not in r.stderr and "runtime error" not in r.stderr, r.stderr[-4000:]
    lines = [ln for ln in r.stdout.splitlines() if ln.startswith("pass")]
    assert len(lines) == 2
    for ln in lines:
        assert "steps 23" in ln  # the tallies restart at the state round trip
        assert " ionized 0 " not in ln and " elastic 0 " not in ln and " wall 0 " not in ln, ln
