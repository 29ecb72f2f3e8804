"""The oracle's CPU pins once more, against a build of the oracle with
AddressSanitizer and UndefinedBehaviorSanitizer (every out-of-bounds
access, use after free, signed overflow, misaligned or null access and
invalid shift aborts the run).  The pins run in a child process that has
libasan preloaded, so that the sanitizer runtime comes before Python's own
allocations; leak checking is off (the interpreter keeps its arenas)."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ORACLE = os.path.join(ROOT, "oracle")
PIN_FILES = ["test_oracle_stream.py", "test_oracle_force.py", "test_oracle_lattice.py",
             "test_oracle_dynamics.py", "test_oracle_adjoint.py", "test_oracle_contact_angle.py",
             "test_oracle_pressure.py", "test_oracle_physics.py"]


def _runtime(name):
    p = subprocess.run(["gcc", "-print-file-name=" + name], capture_output=True, text=True).stdout.strip()
    return p if os.path.isabs(p) and os.path.exists(p) else None


@pytest.mark.slow
def test_oracle_pins_under_asan_and_ubsan(tmp_path):
    asan = _runtime("libasan.so")
    if asan is None:
        pytest.skip("gcc's AddressSanitizer runtime is not installed")
    lib = str(tmp_path / "liboracle_san.so")
    subprocess.run(["make", "-s", "-C", ORACLE, "-f", "sanitize.mk", "-B", "liboracle_san.so"],
                   check=True)
    os.replace(os.path.join(ORACLE, "liboracle_san.so"), lib)
    env = dict(os.environ, LD_PRELOAD=asan, ORACLE_LIB=lib, OMP_NUM_THREADS="8",
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    cmd = [sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", "-m", "not gpu and not slow"]
    cmd += [os.path.join(ROOT, "tests", f) for f in PIN_FILES]
    r = subprocess.run(cmd, cwd=ROOT, env=env, capture_output=True, text=True, timeout=1200)
    tail = "\n".join((r.stdout + r.stderr).splitlines()[-40:])
    assert r.returncode == 0, tail
    assert "passed" in r.stdout and "failed" not in r.stdout, tail
    # the child really ran the sanitized build
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, tail
