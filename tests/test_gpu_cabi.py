"""The library driven from a plain C program (csrc/cabi_demo.c): caller-owned
device memory from the HIP runtime, the calls of include/lbm.h only, no
Python or torch in the process.  The program checks mass conservation, the
limiter bounds of the wall virtual densities and refused out-of-order calls
itself and exits 0 only if all hold."""
import os
import subprocess

import pytest

pytestmark = pytest.mark.gpu


def test_c_program_runs_the_step(gpu_lib):
    from paper_1908_04443_amd import build
    if not os.path.exists(build.DEMO):
        pytest.fail("the C demo is not built (run the package build)")
    r = subprocess.run([build.DEMO], capture_output=True, text=True, timeout=120)
    print(r.stdout, r.stderr, flush=True)
    assert r.returncode == 0
    assert "C ABI demo ok" in r.stdout
