"""The oracle's C code under AddressSanitizer and UndefinedBehaviorSanitizer.

fv_oracle.c is compiled with gcc -fsanitize=address,undefined (no recovery:
the first finding aborts) into a temporary library, and the oracle's CPU pins
(tests/test_oracle.py and tests/test_oracle_local.py) run against it in a
child Python process with the sanitizer runtimes preloaded.  Any
out-of-bounds access, use of uninitialised stack memory by address,
signed overflow or other undefined behaviour in the oracle fails this test.
Host code only: nothing here touches a GPU.
"""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "fv_oracle.c")


def _runtime(name):
    path = subprocess.run(["gcc", "-print-file-name=" + name], capture_output=True,
                          text=True).stdout.strip()
    return path if os.path.isabs(path) and os.path.exists(path) else None


@pytest.mark.slow
def test_oracle_pins_pass_under_asan_and_ubsan(tmp_path):
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    asan, ubsan = _runtime("libasan.so"), _runtime("libubsan.so")
    if not (asan and ubsan):
        pytest.skip("sanitizer runtimes not installed")
    lib = str(tmp_path / "liboracle_san.so")
    cmd = ["gcc", "-O1", "-g", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
           "-fPIC", "-shared", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-o", lib, SRC, "-lm"]
    subprocess.run(cmd, check=True)
    env = dict(os.environ)
    env["FV_ORACLE_LIB"] = lib
    env["LD_PRELOAD"] = asan + ":" + ubsan
    # the interpreter itself is not instrumented: leak reports would be
    # about it, not the oracle
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=1"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    env["OMP_NUM_THREADS"] = "2"
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                        "tests/test_oracle.py", "tests/test_oracle_local.py"],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "runtime error" not in out and "AddressSanitizer" not in out, out[-4000:]
    assert " passed" in out
