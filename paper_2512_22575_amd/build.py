"""Build libsmpc.so (gfx950) in-tree with hipcc.

Usage: ``python -m paper_2512_22575_amd.build`` (or ``build()`` from Python).
The library is written next to this file so that it travels with the source tree.
"""
from __future__ import annotations

import os
import shlex
import subprocess
import sys

PKG_DIR = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG_DIR)
CSRC = os.path.join(PKG_DIR, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB_NAME = "libsmpc.so"
LIB_PATH = os.path.join(PKG_DIR, LIB_NAME)
ARCH = "gfx950"

SOURCES = ["smpc_kernels.hip", "smpc_edt.hip", "smpc_runtime.cpp"]

# Packed FP32 instructions are disabled for device code on purpose (the compiler
# would otherwise form v_pk_* ops from ordinary float code).
DEVICE_FLAGS = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def hipcc() -> str:
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    path = os.path.join(rocm, "bin", "hipcc")
    return path if os.path.exists(path) else "hipcc"


def compile_command(out_path: str = LIB_PATH, extra: list[str] | None = None) -> list[str]:
    return ([hipcc(), f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-shared",
             "-Wall", "-Wshadow", "-Wno-unused-function", f"-I{INCLUDE}", f"-I{CSRC}"] + DEVICE_FLAGS
            + (extra or []) + [os.path.join(CSRC, s) for s in SOURCES] + ["-o", out_path])


def build(verbose: bool = False, out_path: str = LIB_PATH, extra: list[str] | None = None) -> str:
    """Compile every HIP source into ``out_path`` (always recompiles)."""
    cmd = compile_command(out_path, extra)
    if verbose:
        print(" ".join(shlex.quote(c) for c in cmd), flush=True)
    tmp = out_path + ".tmp"
    cmd[-1] = tmp
    res = subprocess.run(cmd, capture_output=True, text=True)
    noise = "is not a recognized feature for this target"
    err = "\n".join(l for l in res.stderr.splitlines() if noise not in l)
    if res.returncode != 0:
        raise RuntimeError(f"hipcc failed ({res.returncode}):\n{err}")
    if verbose and err.strip():
        print(err, file=sys.stderr)
    os.replace(tmp, out_path)
    return out_path


if __name__ == "__main__":
    print(build(verbose=True))
