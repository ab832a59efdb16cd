"""The oracle's pin battery under AddressSanitizer and UBSan.

The oracle source is built once more with -fsanitize=address,undefined
(aborting on the first report) and the pin tests run against that build in
a child process, with the sanitizer runtime loaded first. Any out-of-bounds
access, use after free or undefined arithmetic in the oracle fails the run.
"""
import os
import subprocess
import sys

import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SANITIZE = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined", "-fno-sanitize-recover=all"]


def _runtime(name):
    r = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True)
    path = r.stdout.strip()
    return path if r.returncode == 0 and os.path.isabs(path) and os.path.exists(path) else None


@pytest.mark.timeout(600)
def test_pins_under_asan_and_ubsan(tmp_path):
    asan, ubsan = _runtime("libasan.so"), _runtime("libubsan.so")
    if not asan or not ubsan:
        pytest.skip("gcc sanitizer runtimes not installed")
    lib = oracle.build(path=str(tmp_path / "liboracle_san.so"), flags=SANITIZE)
    env = dict(os.environ)
    env["ET_ORACLE_LIB"] = lib
    env["LD_PRELOAD"] = ":".join(p for p in (asan, ubsan, env.get("LD_PRELOAD", "")) if p)
    # Python itself is not instrumented: its allocations are not leaks of the oracle
    env["ASAN_OPTIONS"] = "detect_leaks=0:verify_asan_link_order=0:abort_on_error=1"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_oracle_pins.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=580)
    tail = (r.stdout + r.stderr)[-4000:]
    assert r.returncode == 0, tail
    assert "ERROR: AddressSanitizer" not in tail and "runtime error" not in tail, tail
