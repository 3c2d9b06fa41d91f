"""Builds the HIP library ``libsgm.so`` (gfx950) in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libsgm.so")
SOURCES = ["sgm_kernels.hip", "sgm_batch.hip", "sgm_server.hip", "sgm_capi.hip", "sgm_static.hip", "sgm_probe.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-shared",
    "-Wall", "-Wno-unused-result",
    # no packed-FP32 instructions anywhere in the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"),
]


def build(verbose: bool = False) -> str:
    """Compile every source into libsgm.so (always recompiles): one hipcc
    process per source in parallel, then one link."""
    objdir = os.path.join(PKG, "_build")
    os.makedirs(objdir, exist_ok=True)
    noise = "is not a recognized feature for this target"
    compile_flags = [f for f in FLAGS if f != "-shared"]
    procs = []
    for src in SOURCES:
        obj = os.path.join(objdir, os.path.splitext(src)[0] + f".{os.getpid()}.o")
        cmd = [HIPCC, *compile_flags, "-c", "-o", obj, os.path.join(CSRC, src)]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((obj, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)))
    msgs, failed = [], False
    for obj, pr in procs:
        out, _ = pr.communicate()
        msgs += [l for l in out.splitlines() if noise not in l and l.strip()]
        failed |= pr.returncode != 0
    tmp = LIB + f".tmp{os.getpid()}"
    if not failed:
        cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *[o for o, _ in procs]]
        if verbose:
            print(" ".join(cmd), flush=True)
        res = subprocess.run(cmd, capture_output=True, text=True)
        msgs += [l for l in (res.stdout + res.stderr).splitlines() if noise not in l and l.strip()]
        failed = res.returncode != 0
    for obj, _ in procs:
        if os.path.exists(obj):
            os.remove(obj)
    if failed:
        raise RuntimeError("hipcc failed:\n" + "\n".join(msgs))
    if msgs and verbose:
        print("\n".join(msgs), file=sys.stderr)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
