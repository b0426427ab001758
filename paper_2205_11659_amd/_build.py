"""Build step for libtreebbox.so (hipcc, gfx950, in-tree)."""
import os
import subprocess

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
LIB = os.path.join(PKG, "libtreebbox.so")
SOURCES = ["csrc/tb_forward.hip", "csrc/tb_api.cpp", "csrc/tb_tune.cpp"]
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
         # never let the compiler form packed fp32 ops
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         # inputs are NaN-free by contract: lets max/min skip NaN quieting
         "-fno-honor-nans",
         # every fp32 product and sum rounds on its own (the fp32 transform
         # payload defines its rounding; nothing else here multiplies and adds)
         "-ffp-contract=off"]


def build(verbose=False):
    tmp = LIB + ".tmp"
    cmd = (["hipcc"] + FLAGS + ["-I" + os.path.join(ROOT, "include"), "-o", tmp]
           + [os.path.join(PKG, s) for s in SOURCES])
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + r.stderr)
    if verbose and r.stderr.strip():
        print(r.stderr)
    os.replace(tmp, LIB)
    return LIB
