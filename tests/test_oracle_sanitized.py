"""The oracle's pin suite, run against a build of qap_oracle.c with AddressSanitizer and
UndefinedBehaviorSanitizer (host code only), so that an out-of-bounds access, an integer
overflow or any other undefined behaviour in the oracle fails the suite instead of
silently changing the values the GPU path is compared with."""
import os
import shutil
import subprocess
import sys
import tempfile

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = os.path.join(ROOT, "oracle", "qap_oracle.c")


def _runtime(name):
    r = subprocess.run(["gcc", "-print-file-name=" + name], capture_output=True, text=True)
    p = r.stdout.strip()
    return p if r.returncode == 0 and os.path.isabs(p) and os.path.exists(p) else None


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc is not installed")
def test_oracle_pins_under_asan_ubsan():
    asan = _runtime("libasan.so")
    if asan is None:
        pytest.skip("no AddressSanitizer runtime for gcc")
    with tempfile.TemporaryDirectory() as tmp:
        lib = os.path.join(tmp, "liboracle_san.so")
        subprocess.check_call(["gcc", "-O1", "-g", "-std=c11", "-Wall", "-Wextra", "-Werror",
                               "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                               "-fno-omit-frame-pointer", "-shared", "-fPIC", SRC, "-o", lib])
        env = dict(os.environ)
        env.update({"QAP_ORACLE_LIB": lib, "LD_PRELOAD": asan,
                    # the interpreter itself is not instrumented: its allocations are not
                    # leaks of the oracle
                    "ASAN_OPTIONS": "detect_leaks=0:abort_on_error=1:verify_asan_link_order=0",
                    "UBSAN_OPTIONS": "print_stacktrace=1:halt_on_error=1"})
        r = subprocess.run([sys.executable, "-m", "pytest", os.path.join(HERE, "test_oracle.py"), "-q",
                            "-m", "not gpu", "-p", "no:cacheprovider", "-W", "ignore::UserWarning"],
                           cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
        out = r.stdout + r.stderr
        assert r.returncode == 0, out[-4000:]
        assert "runtime error" not in out and "AddressSanitizer" not in out, out[-4000:]
        assert " passed" in out
