"""Builds liblmmew.so (the HIP library behind include/lmmew.h) for gfx950, in-tree.

Each source is compiled to an object in parallel (one hipcc per file), then the
objects are linked into the shared library.
"""
import os
import shutil
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "liblmmew.so")
SOURCES = ["kernels.hip", "mlp.hip", "lmmew.hip", "calib.hip"]
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # no packed FP32 instructions anywhere in the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # MFMA results in VGPRs (the fused inference kernel feeds them straight to VALU)
    "-mllvm", "-amdgpu-mfma-vgpr-form",
    "-Wall", "-Wno-unused-function",
]


def hipcc():
    for c in ("/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


def build(verbose=False):
    os.makedirs(OBJ, exist_ok=True)
    cc = hipcc()
    procs = []
    for s in SOURCES:
        obj = os.path.join(OBJ, os.path.splitext(s)[0] + ".o")
        cmd = [cc] + FLAGS + ["-I", os.path.join(ROOT, "include"), "-c", "-o", obj,
                              os.path.join(CSRC, s)]
        procs.append((s, obj, subprocess.Popen(cmd, stdout=subprocess.PIPE,
                                               stderr=subprocess.PIPE, text=True)))
    errs, objs = [], []
    for s, obj, pr in procs:
        out, err = pr.communicate()
        if pr.returncode != 0:
            errs.append(f"{s}:\n{err[-8000:]}")
        elif verbose and err:
            print(err)
        objs.append(obj)
    if errs:
        raise RuntimeError("hipcc failed:\n" + "\n".join(errs))
    tmp = LIB + ".tmp"
    r = subprocess.run([cc, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs,
                       capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + r.stderr[-8000:])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
