"""The NaN-poisoned-LDS debug build (paper_0807_4471_amd.build.build_poison):
its kernels fill the Psi/rho ring with NaN before staging, so a missed halo
row or column turns the result non-finite.  The parity cases of
lds_poison_cases.py (every sweep width, stacked tiles, walls, ragged
lattices, fused and read-out passes, step-wise batches) must match the
oracle with it.  Run in a child process, which loads that library instead
of the regular one."""
import os
import subprocess
import sys

import pytest

from helpers import banner

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_0807_4471_amd", "libsclbm_lds_poison.so")


def test_poisoned_lds_build_matches_oracle():
    if not os.path.exists(LIB):
        pytest.fail(f"{LIB} missing: build it with paper_0807_4471_amd.build.build_poison()")
    banner("NaN-poisoned LDS debug build: parity cases in a child process")
    env = dict(os.environ, SCLBM_LIBRARY=LIB)
    p = subprocess.run([sys.executable, "-u", os.path.join(ROOT, "tests", "lds_poison_cases.py")],
                       env=env, capture_output=True, text=True, timeout=240)
    print(p.stdout[-2000:], p.stderr[-2000:], flush=True)
    assert p.returncode == 0 and p.stdout.strip().startswith("ok")
