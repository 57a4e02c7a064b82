"""Build libsclbm.so (HIP for gfx950) in-tree with hipcc.

    python -m paper_0807_4471_amd.build
"""
from __future__ import annotations

import os
import subprocess
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libsclbm.so")
# (source, extra flags, object name): the kernel file is compiled once per
# storage type so the four kernel sets build in parallel.
UNITS = [("sclbm_kernels.hip", ["-DSCLBM_STORAGE=%d" % k], "sclbm_kernels_s%d.o" % k)
         for k in range(4)] + [("sclbm_dispatch.cpp", [], "sclbm_dispatch.o"),
                               ("sclbm_api.cpp", [], "sclbm_api.o")]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    "-ffp-contract=on",
    # keep the compiler from emitting packed FP32 (v_pk_*_f32) instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
    "-I", os.path.join(ROOT, "include"), "-I", CSRC,
]


# Sources whose code the step kernels are compiled from.
KERNEL_SOURCES = [os.path.join(CSRC, "sclbm_kernels.hip"), os.path.join(CSRC, "sclbm_internal.h")]


def _code_only(text: str) -> str:
    """Source text without comments and with whitespace runs collapsed, so
    that comment and layout edits do not change the hash.  (The kernel
    sources hold no string literal that contains a comment marker.)"""
    import re
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"//[^\n]*", " ", text)
    return " ".join(text.split())


def kernel_source_hash() -> str:
    """Short hash of the code of the kernel sources: identifies the code that
    profiles and counter figures were taken on."""
    import hashlib
    h = hashlib.sha256()
    for path in KERNEL_SOURCES:
        with open(path, encoding="utf-8") as fh:
            h.update(_code_only(fh.read()).encode())
        h.update(b"\0")
    return h.hexdigest()[:16]


# Debug variant: the kernels fill their Psi/rho ring with NaN before staging,
# so a ring cell read without having been staged poisons the result.
POISON_LIB = os.path.join(HERE, "libsclbm_lds_poison.so")


def build(verbose: bool = False, lib: str = LIB, defines=(), subdir: str = "") -> str:
    """Compile the units (in parallel) and link `lib`; `defines` are extra
    preprocessor flags for every unit, `subdir` keeps their objects apart."""
    from concurrent.futures import ThreadPoolExecutor
    t0 = time.time()
    bdir = os.path.join(HERE, "_build", subdir)
    os.makedirs(bdir, exist_ok=True)
    cmds, objs = [], []
    for src, extra, oname in UNITS:
        obj = os.path.join(bdir, oname)
        lang = ["-x", "hip"] if src.endswith(".cpp") else []
        cmds.append([HIPCC, *FLAGS, *defines, *extra, *lang, "-c", os.path.join(CSRC, src),
                     "-o", obj])
        objs.append(obj)
    if verbose:
        for c in cmds:
            print(" ".join(c), flush=True)
    jobs = max(1, min(len(cmds), int(os.environ.get("MAX_JOBS", os.cpu_count() or 1))))
    with ThreadPoolExecutor(jobs) as ex:
        procs = list(ex.map(lambda c: subprocess.run(c, capture_output=True, text=True), cmds))
    for c, p in zip(cmds, procs):
        if p.returncode != 0:
            sys.stderr.write(p.stdout + p.stderr)
            raise subprocess.CalledProcessError(p.returncode, c)
        if verbose and p.stderr.strip():
            # hipcc's host pass does not know the packed-fp32 feature: harmless
            lines = [ln for ln in p.stderr.splitlines() if "packed-fp32-ops" not in ln]
            if lines:
                print("\n".join(lines), flush=True)
    tmp = lib + ".tmp%d" % os.getpid()
    subprocess.check_call([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs])
    os.replace(tmp, lib)
    if verbose:
        print(f"built {lib} in {time.time() - t0:.1f}s", flush=True)
    return lib


CEILING = os.path.join(HERE, "hbm_ceiling")


def build_ceiling(verbose: bool = False) -> str:
    """The bandwidth-ceiling probe (csrc/hbm_ceiling.hip), a stand-alone
    program: plain copy and the step's 18-plane pull with no arithmetic."""
    tmp = CEILING + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "--offload-arch=gfx950", "-O3", "-std=c++17",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           os.path.join(CSRC, "hbm_ceiling.hip"), "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    p = subprocess.run(cmd, capture_output=True, text=True)
    if p.returncode != 0:
        sys.stderr.write(p.stdout + p.stderr)
        raise subprocess.CalledProcessError(p.returncode, cmd)
    os.replace(tmp, CEILING)
    return CEILING


def build_poison(verbose: bool = False) -> str:
    """The NaN-poisoned-LDS debug library (tests only)."""
    return build(verbose, POISON_LIB, ["-DSCLBM_POISON_LDS=1"], "poison")


if __name__ == "__main__":
    build(verbose="-q" not in sys.argv)
    if "--poison" in sys.argv:
        build_poison(verbose="-q" not in sys.argv)
