"""The C ABI from plain C: include/lor.h compiles as C99 with warnings as
errors, a C program links against liblor.so and gets the documented status
codes and messages from host-side argument checks (no GPU needed)."""
import os
import shutil
import subprocess
import tempfile

import pytest

import paper_2210_12253_amd as pkg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_c_client_compiles_links_and_runs():
    pkg.load_library()  # raises if the library has not been built
    libdir = os.path.dirname(pkg.lor.LIB_PATH)
    rocm_lib = os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "lib")
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "abi_from_c")
        cmd = ["gcc", "-std=c99", "-Wall", "-Wextra", "-Werror", "-I", os.path.join(ROOT, "include"),
               os.path.join(ROOT, "tests", "c", "abi_from_c.c"), "-o", exe, "-L", libdir, "-llor",
               f"-Wl,-rpath,{libdir}", f"-Wl,-rpath-link,{rocm_lib}"]
        r = subprocess.run(cmd, capture_output=True, text=True)
        assert r.returncode == 0, r.stderr
        r = subprocess.run([exe], capture_output=True, text=True, timeout=60)
        assert r.returncode == 0, r.stdout + r.stderr
        assert "abi_from_c: ok" in r.stdout
