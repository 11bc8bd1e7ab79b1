"""Host-thread model of the persistent serving launch's protocol (CPU only).

The persistent serving mode is switched off in the library: its launches did
not finish on MI355X.  These tests check on the CPU what the GPU code does
above the memory system: the plan the runtime builds (csrc/plan.cpp, the same
source the library compiles) for the request mixes of the GPU serving tests,
and the ticket / dependency-counter protocol run by threads in place of
workgroups, under ThreadSanitizer (tests/persist_model.cpp).  A model built
with the dependency wait removed must fail, so the checks have teeth."""
import os
import shutil
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
pytestmark = pytest.mark.sanitize


def _build(tmp_path, extra=()):
    if shutil.which("g++") is None:
        pytest.skip("g++ not found")
    exe = str(tmp_path / ("model" + "".join(extra).replace("-D", "_")))
    subprocess.run(["g++", "-std=c++17", "-O1", "-g", "-fsanitize=thread", *extra, "-I",
                    os.path.join(ROOT, "paper_2111_09512_amd", "csrc"), os.path.join(ROOT, "tests", "persist_model.cpp"),
                    os.path.join(ROOT, "paper_2111_09512_amd", "csrc", "plan.cpp"), "-o", exe, "-lpthread"], check=True)
    return exe


def _run(exe, workers, reqs):
    text = f"{workers}\n" + "".join(f"{n} {ops}\n" for n, ops in reqs)
    return subprocess.run([exe], input=text, capture_output=True, text=True, timeout=600,
                          env={**os.environ, "TSAN_OPTIONS": "halt_on_error=1"})


def _ops(outer, mL, mU):
    # one op per sweep: the residual, m_L - 1 L sweeps, m_U - 1 U sweeps, per outer step
    return outer * (1 + (mL - 1) + (mU - 1))


def _mix_of_serving_test():
    """The 60 requests of the GPU mix test (same pool sizes, same generator)."""
    sys.path.insert(0, ROOT)
    from tests.test_gpu_serving import _requests

    class _A:
        def __init__(self, n):
            self.n = n

    pool = [{"A": _A(N ** 3)} for N in (6, 9, 13, 16, 21)]
    return [(pool[r["mid"]]["A"].n, _ops(r["outer"], r["mL"], r["mU"])) for r in _requests(pool, 60, seed=1)]


def test_plan_and_protocol_on_the_serving_mix(tmp_path):
    exe = _build(tmp_path)
    reqs = _mix_of_serving_test()
    for workers in (1024, 64, 7, 1):  # the launch's default cap, and smaller grids
        r = _run(exe, workers, reqs)
        assert r.returncode == 0, r.stdout + r.stderr[-3000:]
        assert "model ok" in r.stdout and "ThreadSanitizer" not in r.stderr


def test_protocol_on_random_mixes(tmp_path):
    exe = _build(tmp_path)
    rng = np.random.default_rng(7)
    for trial in range(4):
        reqs = [(int(rng.integers(1, 300_000)), _ops(int(rng.integers(1, 5)), 3, 3)) for _ in range(int(rng.integers(1, 40)))]
        r = _run(exe, int(rng.integers(1, 200)), reqs)
        assert r.returncode == 0, r.stdout + r.stderr[-3000:]


def test_model_catches_a_missing_wait(tmp_path):
    exe = _build(tmp_path, ("-DPLANT_NO_WAIT",))
    r = _run(exe, 64, _mix_of_serving_test())
    assert r.returncode != 0
    assert "ThreadSanitizer" in r.stderr or "FAIL" in r.stdout
