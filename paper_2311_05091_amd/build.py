"""Builds the HIP libraries libtpf.so and libtpf_nn.so for gfx950 with hipcc
(in-tree).  libtpf.so is compiled from seven translation units in parallel
(the host sides of the 2D and 3D steps and their FP32 and FP64 kernel
instances, and the 3f model) and linked."""
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
FLAGS = ["-O3", "--offload-arch=gfx950", "-std=c++17", "-fPIC",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I", os.path.join(ROOT, "include"), "-I", CSRC]
COMMON = FLAGS + ["-shared"]
LBM_SOURCES = ("tpf_api.hip", "tpf_launch_f32.hip", "tpf_launch_f64.hip", "tpf3_api.hip",
               "tpf3_launch_f32.hip", "tpf3_launch_f64.hip", "tpf3f_api.hip")


def _compile(sources, out, extra=()):
    tmp = out + ".tmp%d" % os.getpid()
    cmd = [HIPCC] + COMMON + list(extra) + list(sources) + ["-o", tmp]
    subprocess.check_call(cmd)
    os.replace(tmp, out)
    return out


def build_lbm() -> str:
    """Compiles the translation units of libtpf.so concurrently, then links."""
    objdir = os.path.join(PKG, "_build")
    os.makedirs(objdir, exist_ok=True)
    procs, objs = [], []
    for src in LBM_SOURCES:
        obj = os.path.join(objdir, src.replace(".hip", ".o"))
        objs.append(obj)
        procs.append(subprocess.Popen([HIPCC] + FLAGS + ["-c", os.path.join(CSRC, src), "-o", obj]))
    failed = [p.args for p in procs if p.wait() != 0]
    if failed:
        raise subprocess.CalledProcessError(1, failed[0])
    tmp = LIB + ".tmp%d" % os.getpid()
    subprocess.check_call([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC"] + objs + ["-o", tmp])
    os.replace(tmp, LIB)
    return LIB


def build_nn() -> str:
    src = os.path.join(CSRC, "tpf_nn.hip")
    if not os.path.exists(src):
        return ""
    return _compile([src], NNLIB)


def build_all():
    """Both libraries; the surrogate library compiles while libtpf.so does."""
    import threading
    res = {}

    def nn():
        try:
            res["nn"] = build_nn()
        except Exception as e:  # re-raised below
            res["err"] = e

    th = threading.Thread(target=nn)
    th.start()
    out = [build_lbm()]
    th.join()
    if "err" in res:
        raise res["err"]
    if res.get("nn"):
        out.append(res["nn"])
    return out


if __name__ == "__main__":
    for p in build_all():
        print(p)
    sys.exit(0)
