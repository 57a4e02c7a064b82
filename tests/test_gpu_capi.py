"""The C ABI alone: tests/capi/capi_check (built by __graft_entry__.build())
allocates device memory with hipMalloc, drives libsclbm.so through
include/sclbm.h only and checks moments against the FP64 totals, the time
counter, two error statuses and a bitwise checkpoint round trip."""
import os
import subprocess

import pytest

from helpers import banner

pytestmark = pytest.mark.gpu

BIN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "capi", "capi_check")


def test_c_program_through_the_abi():
    banner("C program through the C ABI")
    if not os.path.exists(BIN):
        pytest.fail(f"{BIN} is missing: run __graft_entry__.build() first")
    r = subprocess.run([BIN], capture_output=True, text=True, timeout=120)
    print(r.stdout, r.stderr, flush=True)
    assert r.returncode == 0, r.stderr
    assert "capi_check: ok" in r.stdout
