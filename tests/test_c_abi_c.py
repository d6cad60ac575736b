"""The C ABI from plain C: tests/c_abi_host.c is compiled as C99 against
include/fdm.h with gcc (-Wall -Wextra -pedantic -Werror), linked to the
in-tree libfdm.so and run on the host (it uses only entry points that touch
no device: fdm_version, fdm_aca, fdm_last_error, fdm_plan_destroy(NULL))."""
import os
import shutil
import subprocess

import pytest

import paper_2004_14229_amd as F

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not found")
def test_plain_c_client(tmp_path):
    assert os.path.exists(F.LIB_PATH)
    libdir = os.path.dirname(F.LIB_PATH)
    exe = str(tmp_path / "c_abi_host")
    cmd = ["gcc", "-std=c99", "-Wall", "-Wextra", "-pedantic", "-Werror",
           "-I", os.path.join(ROOT, "include"), os.path.join(ROOT, "tests", "c_abi_host.c"),
           "-o", exe, "-L", libdir, "-lfdm", f"-Wl,-rpath,{libdir}",
           "-Wl,-rpath-link,/opt/rocm/lib", "-lm"]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=60)
    assert r.returncode == 0, (r.returncode, r.stdout, r.stderr)
    assert r.stdout.startswith("c abi ok")
