"""Builds libp2p.so (the HIP library behind include/p2p.h) in-tree for gfx950,
and libp2p_issue.so, the VALU issue-rate microbenchmark the benchmark loads.

    python -m paper_2403_01596_amd.build

Each .hip source is compiled with hipcc for gfx950 and the objects are linked
against the HIP runtime that PyTorch loads (so that one runtime serves both the
tensors and the library).  Packed FP32 instructions are turned off for all
device code, and matrix-core instructions keep their accumulators in VGPRs.
"""
from __future__ import annotations

import concurrent.futures
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libp2p.so")
SOURCES = ["api.hip", "memory.hip", "plan.hip", "apply.hip", "backward.hip", "mrhs.hip", "batch.hip",
           "quad2d.hip"]
ISSUE_SOURCES = ["issue_rates.hip"]
ISSUE_LIB = os.path.join(HERE, "libp2p_issue.so")
ARCH = os.environ.get("P2P_OFFLOAD_ARCH", "gfx950")


def hipcc() -> str:
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    return os.path.join(rocm, "bin", "hipcc")


def torch_lib_dir() -> str:
    import torch  # the HIP runtime of the process comes from here

    return os.path.join(os.path.dirname(torch.__file__), "lib")


def compile_flags():
    return ["--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-result",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            # matrix-core accumulators in ordinary VGPRs: the AGPR form made the
            # register allocator copy every accumulator tile each loop trip
            "-mllvm", "-amdgpu-mfma-vgpr-form",
            "-I" + os.path.join(ROOT, "include")]


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    cmd = [hipcc()] + compile_flags() + ["-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc failed for " + src)
    return obj


def _link(objs, lib: str) -> None:
    tl = torch_lib_dir()
    tmp = lib + ".tmp%d" % os.getpid()
    cmd = ["g++", "-shared", "-o", tmp] + objs + ["-L" + tl, "-l:libamdhip64.so", "-Wl,-rpath," + tl,
                                                  "-Wl,--no-undefined"]
    subprocess.check_call(cmd)
    os.replace(tmp, lib)


def build() -> str:
    os.makedirs(BUILD, exist_ok=True)
    with concurrent.futures.ThreadPoolExecutor(max_workers=4) as ex:
        objs = list(ex.map(_compile, SOURCES + ISSUE_SOURCES))
    _link(objs[:len(SOURCES)], LIB)
    _link(objs[len(SOURCES):], ISSUE_LIB)
    return LIB


def device_asm(src: str, out: str) -> None:
    """Writes the gfx950 assembly of one source (for inspection)."""
    cmd = [hipcc()] + compile_flags() + ["--cuda-device-only", "-S", os.path.join(CSRC, src), "-o", out]
    subprocess.check_call(cmd)


if __name__ == "__main__":
    print(build())
