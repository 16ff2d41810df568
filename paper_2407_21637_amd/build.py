"""Build the HIP library ``libhodlr.so`` for gfx950 in-tree.

    python -m paper_2407_21637_amd.build        (or build() from Python)

Compiles ``csrc/host.cpp`` (host core and C ABI) and the device translation
units ``csrc/kernels*.hip`` side by side with hipcc and links them into
``paper_2407_21637_amd/libhodlr.so``, and ``csrc/calibrate.hip`` (the
machine-ceiling probe) into ``paper_2407_21637_amd/calibrate``.  Packed-fp32 instructions are turned
off for the device code (``-packed-fp32-ops``), and MFMA accumulators are
kept in the architectural VGPRs (``-amdgpu-mfma-vgpr-form``): with the
accumulators in AGPRs the compiler copied the leaf GEMM's accumulators
between the two register files on every loop iteration and needed more
registers in total (one wave per SIMD instead of two).
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libhodlr.so")
CALIBRATE = os.path.join(HERE, "calibrate")
ARCH = os.environ.get("HODLR_OFFLOAD_ARCH", "gfx950")

DEVICE_FLAGS = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                "-mllvm", "-amdgpu-mfma-vgpr-form=1"]
# compile-time tuning parameters (hodlr_internal.h, dev_common.h), e.g.
# HODLR_BUILD_DEFINES="HODLR_ITEM_KB=128 HODLR_U_UNROLL=16"
DEFINES = [f"-D{d}" for d in os.environ.get("HODLR_BUILD_DEFINES", "").split() if d]


def _hipcc():
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def _run(cmd):
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if r.returncode != 0:
        sys.stderr.write(" ".join(cmd) + "\n" + r.stdout)
        raise RuntimeError(f"build step failed: {cmd[-1]}")
    return r.stdout


def _run_all(cmds):
    """Run independent compile steps side by side; raise on the first failure."""
    procs = [(c, subprocess.Popen(c, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)) for c in cmds]
    failed = None
    for c, p in procs:
        out, _ = p.communicate()
        if p.returncode != 0 and failed is None:
            failed = (c, out)
    if failed:
        sys.stderr.write(" ".join(failed[0]) + "\n" + failed[1])
        raise RuntimeError(f"build step failed: {failed[0][-1]}")


# device translation units of the library (compiled in parallel)
DEVICE_TUS = ("kernels.hip", "kernels_lowp.hip", "kernels_batch.hip", "kernels_build.hip", "kernels_lu.hip")
HOST_TUS = ("host.cpp", "construct.cpp", "lu.cpp")


def build(verbose: bool = False) -> str:
    hipcc = _hipcc()
    inc = ["-I", os.path.join(ROOT, "include"), "-I", CSRC]
    with tempfile.TemporaryDirectory(prefix="hodlr_build_") as tmp:
        objs, cmds = [], []
        for tu in HOST_TUS:
            o = os.path.join(tmp, tu.replace(".cpp", ".o"))
            objs.append(o)
            cmds.append([hipcc, "-std=c++17", "-O2", "-fPIC", "-Wall", "-c", *DEFINES, *inc,
                         os.path.join(CSRC, tu), "-o", o])
        for tu in DEVICE_TUS:
            o = os.path.join(tmp, tu.replace(".hip", ".o"))
            objs.append(o)
            cmds.append([hipcc, "-std=c++17", "-O3", "-fPIC", f"--offload-arch={ARCH}", *DEVICE_FLAGS, *DEFINES, "-c", *inc,
                         "-x", "hip", os.path.join(CSRC, tu), "-o", o])
        # the machine-ceiling probe (a standalone program, not linked into the library)
        tmp_cal = os.path.join(tmp, "calibrate")
        cmds.append([hipcc, "-std=c++17", "-O3", f"--offload-arch={ARCH}", *DEVICE_FLAGS,
                     os.path.join(CSRC, "calibrate.hip"), "-o", tmp_cal])
        _run_all(cmds)
        tmp_lib = os.path.join(tmp, "libhodlr.so")
        _run([hipcc, "-shared", "-fPIC", f"--offload-arch={ARCH}", *objs, "-o", tmp_lib, "-lpthread"])
        shutil.copyfile(tmp_lib, LIB + ".tmp")
        os.replace(LIB + ".tmp", LIB)
        shutil.copyfile(tmp_cal, CALIBRATE + ".tmp")
        os.chmod(CALIBRATE + ".tmp", 0o755)
        os.replace(CALIBRATE + ".tmp", CALIBRATE)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
