"""The oracle's C code under AddressSanitizer and UBSan: a C driver (tests/sanitize) runs every
mode (plain Shan-Chen with source and merges, barrier, gravity, two components, film geometry,
labelling) in 2D and 3D; any memory or undefined-behaviour error fails the test."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_runs_clean_under_asan_and_ubsan(tmp_path):
    exe = str(tmp_path / "oracle_drive")
    cmd = ["gcc", "-O1", "-g", "-fsanitize=address,undefined", "-fno-omit-frame-pointer",
           "-fno-sanitize-recover=undefined", "-I", os.path.join(ROOT, "oracle"),
           os.path.join(HERE, "sanitize", "oracle_drive.c"),
           os.path.join(ROOT, "oracle", "sc_oracle.c"), "-lm", "-o", exe]
    subprocess.run(cmd, check=True, capture_output=True, timeout=120)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    assert r.returncode == 0, r.stderr[-3000:]
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr
    lines = [l for l in r.stdout.splitlines() if l.startswith("q ")]
    assert len(lines) == 8 and "labels" in r.stdout
