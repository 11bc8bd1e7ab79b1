"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

* The library's host-side set-up (ILU(k), ILUT, the reverse Cuthill-McKee
  order: csrc/factor.cpp, csrc/order.cpp) linked with tests/sanitize_host.cpp
  into one instrumented program, run over valid and rejected inputs, with leak
  detection on.
* The oracle (oracle/oracle.c) built instrumented and every oracle pin test
  run against that build in a child process (the sanitizer runtime preloaded
  into the interpreter, leak detection off since the interpreter itself is not
  instrumented).

Any sanitizer report aborts the program (-fno-sanitize-recover=all), so a pass
means no report was raised."""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g", "-O1"]
ORACLE_TESTS = ["test_oracle_factor.py", "test_oracle_smoother.py", "test_oracle_rowcol.py", "test_oracle_gs.py",
                "test_oracle_krylov.py", "test_oracle_fixed_point.py"]

pytestmark = pytest.mark.sanitize


def _need(tool):
    if shutil.which(tool) is None:
        pytest.skip(f"{tool} not found")


def _runtime(name):
    path = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True).stdout.strip()
    if not os.path.isabs(path) or not os.path.exists(path):
        pytest.skip(f"{name} not installed")
    return path


def test_host_setup_code_sanitized(tmp_path):
    _need("g++")
    _runtime("libasan.so")
    exe = str(tmp_path / "host_san")
    subprocess.run(["g++", "-std=c++17", "-ffp-contract=off", *SAN, "-I", os.path.join(ROOT, "include"),
                    os.path.join(ROOT, "tests", "sanitize_host.cpp"),
                    os.path.join(ROOT, "paper_2111_09512_amd", "csrc", "factor.cpp"),
                    os.path.join(ROOT, "paper_2111_09512_amd", "csrc", "order.cpp"), "-o", exe], check=True)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300,
                       env={**os.environ, "ASAN_OPTIONS": "detect_leaks=1"})
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "all host checks passed" in out
    assert "Sanitizer" not in out and "runtime error" not in out, out[-4000:]


def test_oracle_pins_sanitized(tmp_path):
    _need("gcc")
    asan = _runtime("libasan.so")
    lib = str(tmp_path / "liboracle_san.so")
    subprocess.run(["gcc", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", *SAN,
                    "-o", lib, os.path.join(ROOT, "oracle", "oracle.c"), "-lm"], check=True)
    env = {**os.environ, "ORACLE_LIB": lib, "LD_PRELOAD": asan, "ASAN_OPTIONS": "detect_leaks=0",
           "UBSAN_OPTIONS": "print_stacktrace=1"}
    # the child process confirms it loaded the instrumented build before running the pins
    probe = subprocess.run([sys.executable, "-c", "from oracle import oracle as O; O.lib(); print(O._lib._name)"],
                           cwd=ROOT, env=env, capture_output=True, text=True, timeout=120)
    assert probe.returncode == 0 and probe.stdout.strip() == lib, probe.stdout + probe.stderr
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider", "-m", "not gpu",
                        *[os.path.join("tests", t) for t in ORACLE_TESTS]],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "Sanitizer" not in out and "runtime error" not in out, out[-4000:]
