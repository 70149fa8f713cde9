"""Build libqs.so for gfx950 in-tree with hipcc."""

from __future__ import annotations

import os
import shutil
import subprocess
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libqs.so")

DEVICE_SOURCES = ["qs_kernels.hip"]
HOST_SOURCES = ["qs_runtime.cpp", "qs_plan.cpp"]

# Packed FP32 instructions stay off: hipcc otherwise forms v_pk_* from plain
# float code.
NO_PACKED_FP32 = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]

# MFMA accumulators in ordinary VGPRs: FP32 MFMA and VALU share the SIMD's
# issue cycles on gfx950, so the accumulator-register reads of the AGPR form
# cost matrix time.
MFMA_VGPR = ["-mllvm", "-amdgpu-mfma-vgpr-form"]


def hipcc() -> str:
    return shutil.which("hipcc") or "/opt/rocm/bin/hipcc"


def build(verbose: bool = False, jobs: int = 4) -> str:
    common = ["-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950", "-I", INCLUDE, "-I", CSRC,
              "-Wall", "-Wno-unused-function"]
    # a failed build must not leave an older library behind to be tested
    if os.path.exists(LIB):
        os.remove(LIB)
    tmpdir = tempfile.mkdtemp(prefix="qs_build_")
    objs, procs = [], []
    try:
        for src in DEVICE_SOURCES + HOST_SOURCES:
            obj = os.path.join(tmpdir, src + ".o")
            extra = MFMA_VGPR if src.endswith(".hip") else []
            cmd = [hipcc()] + common + NO_PACKED_FP32 + extra + ["-x", "hip", "-c",
                                                                  os.path.join(CSRC, src), "-o", obj]
            if verbose:
                print(" ".join(cmd), flush=True)
            procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE,
                                                stderr=subprocess.STDOUT, text=True)))
            objs.append(obj)
        for src, p in procs:
            out, _ = p.communicate()
            if p.returncode != 0:
                raise RuntimeError(f"hipcc failed on {src}:\n{out}")
            if verbose and out.strip():
                print(out)
        tmp_lib = LIB + ".tmp"
        cmd = [hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp_lib] + objs
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
        os.replace(tmp_lib, LIB)
    finally:
        shutil.rmtree(tmpdir, ignore_errors=True)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
