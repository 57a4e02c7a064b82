"""The oracle and the host side of libsclbm.so under AddressSanitizer and
UndefinedBehaviorSanitizer (CPU only; sanitizers instrument host code
alone, the kernels are linked from the regular build).

tests/sanitize/oracle_check.c drives every oracle entry point on periodic
and walled lattices, both force couplings, one-row and one-column lattices
and the invalid-argument paths; tests/sanitize/host_check.c drives every
host path of the library that does no device work (validation, binding,
tilings, checkpoint headers, batch sizing and refusals, the static-scratch
batch's refusals).  Either program aborts on the first sanitizer report,
leaks included."""
import glob
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = os.path.join(ROOT, "tests", "sanitize")
CSRC = os.path.join(ROOT, "paper_0807_4471_amd", "csrc")
KERNEL_OBJS = sorted(glob.glob(os.path.join(ROOT, "paper_0807_4471_amd", "_build",
                                            "sclbm_kernels_s*.o")))
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1",
           UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
HOST_SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer"]


def _run(cmd, **kw):
    p = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert p.returncode == 0, f"{' '.join(cmd)}\n{p.stdout}\n{p.stderr}"
    return p


def test_oracle_clean_under_asan_ubsan(tmp_path):
    exe = str(tmp_path / "oracle_check")
    _run(["gcc", "-std=c99", "-O1", "-g", "-fsanitize=address,undefined",
          "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-fopenmp",
          "-I", os.path.join(ROOT, "oracle"), os.path.join(SAN, "oracle_check.c"),
          os.path.join(ROOT, "oracle", "sclbm_oracle.c"), "-lm", "-o", exe])
    p = _run([exe], env=ENV, timeout=300)
    assert p.stdout.strip() == "ok"


@pytest.mark.skipif(len(KERNEL_OBJS) != 4 or not shutil.which("/opt/rocm/bin/hipcc"),
                    reason="needs the kernel objects of paper_0807_4471_amd.build and hipcc")
def test_host_runtime_clean_under_asan_ubsan(tmp_path):
    hipcc = ["/opt/rocm/bin/hipcc", "-x", "hip", "--offload-arch=gfx950", "-std=c++17", "-O1",
             "-g", "-fPIC", *HOST_SAN, "-I", os.path.join(ROOT, "include"), "-I", CSRC]
    objs = []
    for src in ("sclbm_api.cpp", "sclbm_dispatch.cpp"):
        o = str(tmp_path / (src + ".o"))
        _run([*hipcc, "-c", os.path.join(CSRC, src), "-o", o])
        objs.append(o)
    clang = "/opt/rocm/llvm/bin/clang"
    drv = str(tmp_path / "host_check.o")
    _run([clang, "-std=c99", "-O1", "-g", "-fsanitize=address,undefined",
          "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-D__HIP_PLATFORM_AMD__",
          "-I", os.path.join(ROOT, "include"), "-I", "/opt/rocm/include",
          "-c", os.path.join(SAN, "host_check.c"), "-o", drv])
    exe = str(tmp_path / "host_check")
    _run([clang + "++", "-fsanitize=address,undefined", "-o", exe, drv, *objs, *KERNEL_OBJS,
          "-L/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib"])
    p = _run([exe], env=ENV, timeout=300)
    assert p.stdout.strip() == "ok"
