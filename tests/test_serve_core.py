"""Host-only checks under AddressSanitizer and UndefinedBehaviorSanitizer:

* the request server's scheduling core (csrc/serve_core.h: admission,
  merging, table budget, slot reuse, release rules, failures, a randomised
  run with invariants) driven by a fake executor (tests/native/
  serve_core_check.cpp), built with g++;
* every oracle pin test (tests/test_oracle_*.py) rerun against an oracle
  library built with the sanitizers, in a subprocess that preloads the ASan
  runtime."""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.dirname(os.path.abspath(__file__))
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer", "-g"]

pytestmark = pytest.mark.skipif(shutil.which("g++") is None or shutil.which("gcc") is None,
                                reason="needs the host compilers")


def test_serve_core_with_fake_executor(tmp_path):
    exe = str(tmp_path / "serve_core_check")
    subprocess.check_call(["g++", "-std=c++17", "-O1", "-Wall", "-Wextra", *SAN,
                           "-I", os.path.join(ROOT, "paper_2010_01775_amd", "csrc"),
                           os.path.join(HERE, "native", "serve_core_check.cpp"), "-o", exe])
    out = subprocess.run([exe], capture_output=True, text=True, timeout=300,
                         env={**os.environ, "ASAN_OPTIONS": "detect_leaks=1:abort_on_error=0"})
    assert out.returncode == 0, out.stderr[-4000:]
    assert out.stdout.strip() == "ok"


def test_oracle_pins_under_sanitizers():
    asan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    if not os.path.isabs(asan) or not os.path.exists(asan):
        pytest.skip("the ASan runtime library is not installed")
    env = {**os.environ, "NPG_ORACLE_SANITIZE": "1", "LD_PRELOAD": asan,
           "ASAN_OPTIONS": "detect_leaks=0:abort_on_error=0", "UBSAN_OPTIONS": "print_stacktrace=1"}
    tests = sorted(os.path.join(HERE, f) for f in os.listdir(HERE)
                   if f.startswith("test_oracle_") and f.endswith(".py"))
    out = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider", "-m", "not gpu",
                          *tests], capture_output=True, text=True, timeout=900, env=env, cwd=ROOT)
    assert out.returncode == 0, (out.stdout[-3000:], out.stderr[-3000:])
    assert "passed" in out.stdout
