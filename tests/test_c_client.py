"""The C ABI from a plain C99 client (tests/c/abi_client.c): include/rsc.h compiles as
strict C (gcc -std=c99 -pedantic -Werror) and as C++, and the client, linked against
librsc.so, checks the host-only calls against values the paper and the mathematics fix
(disk pixel counts, B, the annular cut-offs, Phi^+ Phi = I) and the argument errors.
Needs no GPU."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
INC = os.path.join(ROOT, "include")
SRC = os.path.join(ROOT, "tests", "c", "abi_client.c")


def _lib_dir():
    from paper_1806_04374_amd import rsc
    if not os.path.exists(rsc.LIB_PATH):
        pytest.skip("librsc.so is not built")
    return os.path.dirname(rsc.LIB_PATH)


@pytest.mark.skipif(shutil.which("gcc") is None, reason="no gcc")
def test_c_client(tmp_path):
    lib = _lib_dir()
    exe = str(tmp_path / "abi_client")
    cmd = ["gcc", "-std=c99", "-pedantic", "-Wall", "-Wextra", "-Werror", "-I", INC, SRC, "-o", exe,
           "-L", lib, "-lrsc", f"-Wl,-rpath,{lib}", "-lm"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    print(r.stdout)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "FAIL" not in r.stdout and r.stdout.count("ok  ") == 13


@pytest.mark.skipif(shutil.which("g++") is None, reason="no g++")
def test_header_compiles_as_cpp(tmp_path):
    src = tmp_path / "h.cpp"
    src.write_text('#include "rsc.h"\nstatic_assert(sizeof(rsc_status) == sizeof(int), "enum size");\n'
                   'rsc_status (*const probe)(rsc_handle*) = &rsc_destroy;\n')
    r = subprocess.run(["g++", "-std=c++17", "-Wall", "-Wextra", "-Werror", "-pedantic", "-fsyntax-only", "-I", INC,
                        str(src)], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
