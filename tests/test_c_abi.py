"""The C ABI from plain C99: include/kappa.h compiles with gcc -std=c99
-pedantic -Werror and no HIP headers, a C program links against libkappa.so
and its GPU-free calls (setup, validation, status strings) behave as the
header documents."""
import os
import shutil
import subprocess

import pytest

from paper_2602_05606_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not installed")
def test_plain_c_program(tmp_path):
    exe = tmp_path / "abi_from_c"
    lib_dir = os.path.dirname(_lib.LIB_PATH)
    cmd = ["gcc", "-std=c99", "-Wall", "-Wextra", "-pedantic", "-Werror",
           "-I", os.path.join(ROOT, "include"), os.path.join(ROOT, "tests", "c", "abi_from_c.c"),
           "-L", lib_dir, "-lkappa", f"-Wl,-rpath,{lib_dir}", "-lm", "-o", str(exe)]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    res = subprocess.run([str(exe)], capture_output=True, text=True, timeout=60)
    assert res.returncode == 0, res.stdout + res.stderr
    assert res.stdout.startswith("ok")
