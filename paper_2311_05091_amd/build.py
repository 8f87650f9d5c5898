"""Builds the HIP library libtpf.so for gfx950 with hipcc (in-tree)."""
from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libtpf.so")
NNLIB = os.path.join(PKG, "libtpf_nn.so")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
# packed FP32 instructions are disabled on purpose: the compiler must not form
# v_pk_* FP32 operations
COMMON = ["-O3", "--offload-arch=gfx950", "-std=c++17", "-fPIC", "-shared",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-I", os.path.join(ROOT, "include"), "-I", CSRC]


def _compile(sources, out, extra=()):
    tmp = out + ".tmp%d" % os.getpid()
    cmd = [HIPCC] + COMMON + list(extra) + list(sources) + ["-o", tmp]
    subprocess.check_call(cmd)
    os.replace(tmp, out)
    return out


def build_lbm() -> str:
    return _compile([os.path.join(CSRC, "tpf_api.hip")], LIB)


def build_nn() -> str:
    src = os.path.join(CSRC, "tpf_nn.hip")
    if not os.path.exists(src):
        return ""
    return _compile([src], NNLIB)


def build_all():
    out = [build_lbm()]
    nn = build_nn()
    if nn:
        out.append(nn)
    return out


if __name__ == "__main__":
    for p in build_all():
        print(p)
    sys.exit(0)
