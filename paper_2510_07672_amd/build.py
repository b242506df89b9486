"""Compile libpr.so (the HIP kernels and the C ABI) for gfx950, in tree."""

from __future__ import annotations

import os
import shutil
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libpr.so")
SOURCES = ["api.hip", "fine_kernels.hip", "cnn_kernels.hip", "loss_kernels.hip"]

HIPCC_FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    # no packed-FP32 instructions: plain scalar float arithmetic only
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # fuse multiply-adds only within one source expression, so the same
    # inline arithmetic rounds identically in every kernel that uses it
    "-ffp-contract=on",
    "-Wall",
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found: the ROCm toolchain is required to build libpr")


def build(verbose: bool = False) -> str:
    """Compile every HIP source (in parallel, one object each) and link them
    into paper_2510_07672_amd/libpr.so."""
    import tempfile
    with tempfile.TemporaryDirectory(prefix="libpr_") as tmpd:
        procs, objs = [], []
        for src in SOURCES:
            obj = os.path.join(tmpd, src.replace(".hip", ".o"))
            cmd = [hipcc(), *HIPCC_FLAGS, "-c", "-o", obj, os.path.join(CSRC, src)]
            procs.append((cmd, subprocess.Popen(cmd, cwd=CSRC, stdout=subprocess.PIPE,
                                                stderr=subprocess.STDOUT, text=True)))
            objs.append(obj)
        logs = []
        for cmd, pr in procs:
            out, _ = pr.communicate()
            if pr.returncode != 0:
                raise RuntimeError("hipcc failed:\n" + " ".join(cmd) + "\n" + out)
            logs.append(out)
        tmp = LIB + ".tmp"
        cmd = [hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs
        proc = subprocess.run(cmd, cwd=CSRC, capture_output=True, text=True)
        if proc.returncode != 0:
            raise RuntimeError("link failed:\n" + " ".join(cmd) + "\n" + proc.stdout + proc.stderr)
        if verbose:
            print("".join(logs) + proc.stdout + proc.stderr)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
