"""The C-ABI from plain C99 (CPU only): the public headers compile as C with
warnings as errors, a program links against the library, and the host entry
points (the relabeling order, host ILU(0), status strings) work from C."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIBDIR = os.path.join(ROOT, "paper_2111_09512_amd")


@pytest.mark.skipif(shutil.which("gcc") is None, reason="no C compiler")
def test_headers_compile_as_c99_and_host_entry_points_run(tmp_path):
    lib = os.path.join(LIBDIR, "libscaledilu.so")
    if not os.path.exists(lib):
        pytest.skip("library not built")
    exe = str(tmp_path / "c_abi_host")
    subprocess.run(["gcc", "-std=c99", "-Wall", "-Wextra", "-Werror", "-I", os.path.join(ROOT, "include"),
                    os.path.join(ROOT, "tests", "c_abi_host.c"), "-L", LIBDIR, "-lscaledilu",
                    "-Wl,-rpath," + LIBDIR, "-o", exe], check=True, capture_output=True, text=True)
    out = subprocess.run([exe], capture_output=True, text=True, timeout=60)
    assert out.returncode == 0, out.stdout + out.stderr
    assert "c-abi ok" in out.stdout
