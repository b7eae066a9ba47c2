"""The CPU oracle and the input generator under AddressSanitizer and
UndefinedBehaviorSanitizer: both C sources are rebuilt with
-fsanitize=address,undefined (host code only) and the oracle's pins run
against those builds in a child process, which fails on the first report."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _runtime(name):
    path = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True).stdout.strip()
    return path if os.path.isabs(path) and os.path.exists(path) else None


@pytest.mark.timeout(900)
def test_oracle_and_generator_under_asan_ubsan(tmp_path):
    asan = _runtime("libasan.so")
    if asan is None:
        pytest.skip("gcc has no AddressSanitizer runtime here")
    flags = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
             "-fno-sanitize-recover=undefined", "-fPIC", "-shared", "-ffp-contract=off", "-std=c11"]
    libs = {}
    for name, src, extra in (("ORACLE_LIB_PATH", "oracle/oracle.c", []),
                             ("SYNTH_LIB_PATH", "synth/synth.c", ["-fopenmp"])):
        out = str(tmp_path / (os.path.basename(src)[:-2] + "_san.so"))
        subprocess.run(["gcc", *flags, *extra, "-o", out, os.path.join(ROOT, src), "-lm"], check=True)
        libs[name] = out
    env = dict(os.environ, **libs)
    env["LD_PRELOAD"] = asan
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=1:halt_on_error=1"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", "-m", "not gpu",
                        os.path.join(ROOT, "tests", "test_oracle_pins.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=850)
    tail = (r.stdout + r.stderr)[-3000:]
    assert r.returncode == 0, tail
    assert "ERROR: AddressSanitizer" not in tail and "runtime error" not in tail, tail
