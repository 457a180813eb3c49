"""The boundary is a C ABI: a plain C99 program (tests/c/abi_host.c)
compiled with gcc against include/lbm.h and linked with liblbm.so runs the
host-side calls (argument checks, call order, geometry, node classes)
without a GPU.  Its solid count equals a brute-force count of the closed
disk."""
import os
import shutil
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIBDIR = os.path.join(ROOT, "paper_2605_30878_amd")


@pytest.mark.skipif(shutil.which("gcc") is None, reason="no C compiler")
def test_header_compiles_as_c_and_host_calls_run(tmp_path):
    if not os.path.exists(os.path.join(LIBDIR, "liblbm.so")):
        pytest.skip("library not built")
    exe = str(tmp_path / "abi_host")
    cmd = ["gcc", "-std=c99", "-Wall", "-Wextra", "-Werror", "-pedantic", "-I", os.path.join(ROOT, "include"),
           os.path.join(ROOT, "tests", "c", "abi_host.c"), "-L", LIBDIR, "-llbm", "-Wl,-rpath," + LIBDIR,
           "-o", exe]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    res = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert res.returncode == 0, res.stderr
    words = res.stdout.split()
    counts = dict(zip(words[0::2], words[1::2]))
    y, x = np.mgrid[0:48, 0:64]
    assert int(counts["solid"]) == int(((x - 32.0) ** 2 + (y - 20.0) ** 2 <= 9.5 ** 2).sum())
    assert int(counts["ghost"]) > 0 and int(counts["near"]) > 0 and int(counts["device_bytes"]) > 0
