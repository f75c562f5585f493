"""The oracle's pins again on an AddressSanitizer + UndefinedBehaviorSanitizer
build of the oracle (CPU only): every out-of-bounds access, use after free
or undefined operation in es_oracle.c that the pins exercise stops the run.
The pins run in a child process with the sanitizer runtime preloaded."""
import os
import subprocess
import sys

import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PINS = ["tests/test_oracle_pointwise.py", "tests/test_oracle_sign.py", "tests/test_oracle_bc.py",
        "tests/test_oracle_stage_mesh.py", "tests/test_oracle_monitor_vars.py"]


def test_oracle_pins_clean_under_asan_and_ubsan(tmp_path):
    asan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    if not os.path.isabs(asan) or not os.path.exists(asan):
        pytest.skip("gcc's AddressSanitizer runtime is not installed")
    lib = oracle.build(out=str(tmp_path / "liboracle_san.so"), sanitize=True)
    env = dict(os.environ, ES_ORACLE_LIB=lib, LD_PRELOAD=asan, OMP_NUM_THREADS="2",
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=0:exitcode=86",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1:exitcode=87")
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider", *PINS],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    out = r.stdout + r.stderr
    assert "AddressSanitizer" not in out and "runtime error" not in out, out[-4000:]
    assert r.returncode == 0, out[-4000:]
