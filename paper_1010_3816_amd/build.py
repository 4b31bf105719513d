"""Compile libteuk.so for gfx950 with hipcc (in-tree, no JIT cache)."""
import os
import subprocess

PKG = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libteuk.so")
SOURCES = ["lw_kernels.hip", "adjoint_kernels.hip", "teuk_api.cpp"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

# -packed-fp32-ops: no packed FP32 instructions are generated (all arithmetic
# here is FP64 anyway).  -ffp-contract=on: a multiply and an add are fused
# only within one source expression, never across statements, so code shared
# by several kernels rounds the same way in each of them (the one-step,
# two-step and batched kernels give bit-identical results).
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared", "-Wall", "-ffp-contract=on",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-x", "hip"]


def build(extra=(), out=None):
    lib = out or LIB
    tmp = lib + ".tmp"
    cmd = [HIPCC, *FLAGS, *extra, *[os.path.join(CSRC, s) for s in SOURCES], "-o", tmp]
    print("+", " ".join(cmd), flush=True)
    r = subprocess.run(cmd, cwd=PKG, capture_output=True, text=True)
    noise = "is not a recognized feature for this target"
    msg = "\n".join(l for l in (r.stdout + r.stderr).splitlines() if noise not in l)
    if msg.strip():
        print(msg, flush=True)
    if r.returncode != 0:
        raise subprocess.CalledProcessError(r.returncode, cmd)
    os.replace(tmp, lib)
    return lib


if __name__ == "__main__":
    build()
