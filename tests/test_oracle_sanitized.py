"""The oracle under AddressSanitizer and UndefinedBehaviorSanitizer (host only, CPU): a small C
driver runs every entry point (threaded propagation of both atomic potentials with a non-finite
sample, dipole, resampling, spectrum, one recorded trajectory, the contract functions on awkward
arguments); the sanitized build must report nothing and print exactly what the plain build does."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = [os.path.join(HERE, "oracle_sanitize_driver.c"), os.path.join(ROOT, "oracle", "sfhk_oracle.c")]
BASE = ["-std=gnu11", "-mfma", "-ffp-contract=off", "-fno-fast-math", "-Wall",
        "-Wno-unused-function"]
LIBS = ["-lquadmath", "-lm", "-lpthread"]


def _build_and_run(tmp_path, name, flags):
    exe = str(tmp_path / name)
    subprocess.run(["gcc", *BASE, *flags, "-o", exe, *SRC, *LIBS], check=True,
                   capture_output=True, text=True)
    # verify_asan_link_order=0: the sanitizer runtime need not come first among the loaded libraries
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    return r


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_oracle_clean_under_asan_and_ubsan(tmp_path):
    plain = _build_and_run(tmp_path, "plain", ["-O2"])
    assert plain.returncode == 0, plain.stderr
    san = _build_and_run(tmp_path, "san", ["-O1", "-g", "-fno-omit-frame-pointer",
                                           "-fsanitize=address,undefined",
                                           "-fno-sanitize-recover=all"])
    assert san.returncode == 0, san.stderr[-4000:]
    assert "runtime error" not in san.stderr and "AddressSanitizer" not in san.stderr, san.stderr
    assert san.stdout == plain.stdout
    lines = plain.stdout.splitlines()
    assert lines[0].startswith("softcore") and lines[1].startswith("screened")
    assert "nonfinite=1" in lines[0] and "nonfinite=1" in lines[1]
