"""The C ABI used from plain C99 (no Python, no torch): headers compile with
-std=c99 -pedantic -Werror, the library links, and host-side calls behave
as the headers document.  No device is needed."""
import os
import shutil
import subprocess

import pytest

from paper_1701_08547_amd import api

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("gcc") is None, reason="no C compiler")
def test_c99_host_program(tmp_path):
    if not os.path.exists(api.LIB_PATH):
        pytest.skip("library not built")
    lib_dir = os.path.dirname(api.LIB_PATH)
    exe = tmp_path / "abi_host"
    subprocess.run(["gcc", "-std=c99", "-Wall", "-Wextra", "-pedantic", "-Werror", "-I", os.path.join(ROOT, "include"),
                    os.path.join(ROOT, "tests", "c", "abi_host.c"), "-L", lib_dir, "-lsa",
                    "-Wl,-rpath," + lib_dir, "-o", str(exe)], check=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    assert r.stdout.strip() == "ok"
