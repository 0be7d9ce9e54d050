"""The C oracle under AddressSanitizer and UndefinedBehaviorSanitizer: a
driver (tests/oracle_asan_main.c) linked with oracle/oracle.c calls every
exported function on small and degenerate inputs with exactly sized
buffers; an out-of-bounds access, a leak or undefined arithmetic anywhere in
the oracle ends the run with an error, as does a failed invariant."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not found")
def test_oracle_clean_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_asan")
    cmd = ["gcc", "-O1", "-g", "-std=c11", "-fopenmp", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-Wall", "-Wextra",
           "-o", exe, os.path.join(HERE, "oracle_asan_main.c"),
           os.path.join(ROOT, "oracle", "oracle.c"), "-lm"]
    subprocess.run(cmd, check=True)
    env = dict(os.environ)
    env["ASAN_OPTIONS"] = "detect_leaks=1:abort_on_error=0:halt_on_error=1:verify_asan_link_order=0"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    r = subprocess.run([exe], env=env, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-4000:]
    assert "oracle sanitizer run ok" in r.stdout
    assert "runtime error" not in r.stderr, r.stderr[-4000:]
