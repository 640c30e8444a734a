"""Builds libssm_cascade.so from csrc/ with hipcc for gfx950.

Every source is compiled to an object with ``hipcc --offload-arch=gfx950``
and the objects are linked into a shared library next to this file. The
library is linked against the HIP runtime that PyTorch ships when PyTorch is
installed, so that a process which imports torch first maps a single HIP
runtime (torch's) and torch streams and allocations can be handed to it.
"""

from __future__ import annotations

import concurrent.futures
import glob
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB_NAME = "libssm_cascade.so"
LIB_PATH = os.path.join(HERE, LIB_NAME)
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
ARCH = "gfx950"

HIPCC_FLAGS = [
    f"--offload-arch={ARCH}",
    "-O3",
    "-fPIC",
    "-std=c++17",
    "-Wall",
    "-Wno-unused-function",
    # packed FP32 instructions are kept out of every kernel
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def _torch_lib_dir():
    try:
        import importlib.util

        spec = importlib.util.find_spec("torch")
        if spec is None or spec.origin is None:
            return None
        d = os.path.join(os.path.dirname(spec.origin), "lib")
        return d if os.path.exists(os.path.join(d, "libamdhip64.so")) else None
    except Exception:
        return None


def _compile(src, obj):
    cmd = [os.path.join(ROCM, "bin", "hipcc"), "-c", *HIPCC_FLAGS, src, "-o", obj]
    if src.endswith(".cpp"):
        cmd[2:2] = ["-x", "hip"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    noise = "'-packed-fp32-ops' is not a recognized feature"
    msg = "\n".join(l for l in (r.stdout + r.stderr).splitlines() if noise not in l)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {os.path.basename(src)}:\n{msg}")
    return msg


def build(verbose=False, out=LIB_PATH):
    """Compile all of csrc/ and link ``out``. Always rebuilds."""
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")) + glob.glob(os.path.join(CSRC, "*.cpp")))
    if not srcs:
        raise RuntimeError("no sources under " + CSRC)
    bdir = os.path.join(HERE, "_build")
    os.makedirs(bdir, exist_ok=True)
    objs = [os.path.join(bdir, os.path.basename(s) + ".o") for s in srcs]
    workers = min(len(srcs), max(1, min(8, os.cpu_count() or 1)))
    with concurrent.futures.ThreadPoolExecutor(workers) as ex:
        for src, msg in zip(srcs, ex.map(_compile, srcs, objs)):
            if verbose and msg.strip():
                print(f"[{os.path.basename(src)}]\n{msg}", file=sys.stderr)
    tlib = _torch_lib_dir()
    if tlib:
        link = ["-L" + tlib, "-l:libamdhip64.so", "-Wl,-rpath," + tlib]
    else:
        link = ["-L" + os.path.join(ROCM, "lib"), "-lamdhip64", "-Wl,-rpath," + os.path.join(ROCM, "lib")]
    clang = os.path.join(ROCM, "lib", "llvm", "bin", "clang++")
    if not os.path.exists(clang):
        clang = shutil.which("clang++") or "g++"
    tmp = out + ".tmp"
    cmd = [clang, "-shared", "-o", tmp, *objs, *link, "-Wl,--no-undefined", "-lstdc++", "-lm"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + r.stdout + r.stderr)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose=True))
