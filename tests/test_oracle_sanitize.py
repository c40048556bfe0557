"""The oracle's C sources built with gcc's AddressSanitizer and UndefinedBehaviorSanitizer
(CPU only) and run on the inputs of `oracle_sanitize.c`: no memory or undefined-behaviour
report, and the documented return code for every input."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ORACLE = os.path.join(os.path.dirname(HERE), "oracle")
SOURCES = ["exact.c", "predicates.c", "moore.c", "delaunay.c"]


def test_oracle_under_sanitizers(tmp_path):
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("gcc not found")
    exe = str(tmp_path / "oracle_sanitize")
    cmd = [gcc, "-O1", "-g", "-ffp-contract=off", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=undefined", "-I", ORACLE, os.path.join(HERE, "oracle_sanitize.c")]
    cmd += [os.path.join(ORACLE, s) for s in SOURCES] + ["-lm", "-o", exe]
    b = subprocess.run(cmd, capture_output=True, text=True, timeout=300)
    if b.returncode != 0 and "asan" in b.stderr.lower():
        pytest.skip("sanitizer runtime not available: " + b.stderr[-300:])
    assert b.returncode == 0, b.stderr
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300,
                       env=dict(os.environ, ASAN_OPTIONS="detect_leaks=1"))
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    assert r.stdout.rstrip().endswith("done")
    assert "ERROR" not in r.stderr and "runtime error" not in r.stderr
