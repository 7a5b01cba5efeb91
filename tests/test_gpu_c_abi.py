"""The library called from plain C99 (tests/c_abi_demo.c): HIP runtime C API
for device memory, lightfuse.h for everything else, no Python marshalling.
Checks a closed-form single-surfel case forward and backward.  Requires an
MI355X."""
import os
import subprocess

import pytest

from tests.test_abi import compile_c_demo

pytestmark = pytest.mark.gpu


def test_c_caller_forward_and_backward(tmp_path):
    exe = compile_c_demo(tmp_path)
    print("running", exe, flush=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, (r.returncode, r.stdout, r.stderr)
    assert "c abi ok" in r.stdout, r.stdout
