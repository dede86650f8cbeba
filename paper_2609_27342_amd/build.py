"""Build libtlmpm.so (gfx950) in-tree with hipcc."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libtlmpm.so")
SOURCES = [os.path.join(CSRC, "tlmpm_kernels.hip"), os.path.join(CSRC, "tlmpm_contact.hip"),
           os.path.join(CSRC, "tlmpm_quad.hip"), os.path.join(CSRC, "tlmpm_surface.hip"),
           os.path.join(CSRC, "tlmpm_capi.cpp")]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = ["-O3", "-std=c++17", "-fPIC", "-shared", "--offload-arch=gfx950",
         # multiply-adds fuse only within one source expression, so every kernel
         # wrapper around a shared body rounds the same way (bitwise-equal results
         # for one scene and for a batch)
         "-ffp-contract=on",
         # packed FP32 instructions stay off: ordinary float code only
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-function", "-Wno-unused-variable"]


def build(force=True, verbose=False):
    newest = max(os.path.getmtime(p) for p in SOURCES + [os.path.join(CSRC, "tlmpm_common.h"),
                                                          os.path.join(CSRC, "tlmpm_device.h"),
                                                          os.path.join(CSRC, "tlmpm_band.h"),
                                                          os.path.join(CSRC, "tlmpm_reach.h"),
                                                          os.path.join(HERE, "..", "include", "tlmpm.h")])
    if not force and os.path.exists(LIB) and os.path.getmtime(LIB) >= newest:
        return LIB
    tmp = LIB + ".tmp"
    cmd = [HIPCC] + FLAGS + ["-o", tmp] + SOURCES
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
