"""The oracle's C code under AddressSanitizer and UndefinedBehaviorSanitizer.

The oracle pin tests run in a subprocess against a sanitized build of the
same source (gcc, the sanitizer runtimes preloaded into the interpreter, which
is not itself instrumented).  Any sanitizer report fails the test: an
out-of-bounds access, a use after free or undefined behaviour in the oracle
would make every parity comparison against it suspect."""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "stencil_oracle.c")
PINS = os.path.join(ROOT, "tests", "test_oracle_pins.py")


def _runtime(gcc: str, name: str) -> str:
    path = subprocess.run([gcc, f"-print-file-name={name}"], capture_output=True, text=True).stdout.strip()
    return path if os.path.isabs(path) and os.path.exists(path) else ""


def test_oracle_pins_under_address_and_ub_sanitizers(tmp_path):
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("gcc is not available")
    asan, ubsan = _runtime(gcc, "libasan.so"), _runtime(gcc, "libubsan.so")
    if not asan or not ubsan:
        pytest.skip("the gcc sanitizer runtimes are not installed")
    lib = str(tmp_path / "liboracle_sanitized.so")
    subprocess.run([gcc, "-std=c11", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                    "-fno-sanitize-recover=undefined", "-fopenmp", "-fPIC", "-shared", "-Wall", "-Wextra", "-o", lib,
                    SRC, "-lm"], check=True)
    # reports go to log files: a sanitizer abort would lose what the child's
    # pytest holds in its capture
    logs = tmp_path / "san"
    env = dict(os.environ, LD_PRELOAD=f"{asan}:{ubsan}", OMP_NUM_THREADS="2",
               ASAN_OPTIONS=f"detect_leaks=0:verify_asan_link_order=0:log_path={logs}",
               UBSAN_OPTIONS=f"print_stacktrace=1:halt_on_error=1:log_path={logs}")
    driver = ("import sys, oracle, pytest; oracle.use_library(sys.argv[1]); "
              "sys.exit(pytest.main(['-q', '-x', '-s', '-p', 'no:cacheprovider', sys.argv[2]]))")
    r = subprocess.run([sys.executable, "-c", driver, lib, PINS], cwd=ROOT, env=env, capture_output=True,
                       text=True, timeout=1200)
    reports = "".join(open(os.path.join(tmp_path, f)).read() for f in sorted(os.listdir(tmp_path))
                      if f.startswith("san"))
    out = r.stdout + r.stderr
    assert not reports, reports[:4000]
    assert "AddressSanitizer" not in out and "runtime error" not in out, out[-4000:]
    assert r.returncode == 0, out[-4000:]
    assert " passed" in r.stdout, out[-2000:]
