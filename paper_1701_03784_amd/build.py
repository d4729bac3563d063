"""Builds the HIP library libaxpic.so for gfx950 in-tree (hipcc)."""

from __future__ import annotations

import concurrent.futures as cf
import glob
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT_DIR = os.path.join(HERE, "_lib")
LIB = os.path.join(OUT_DIR, "libaxpic.so")
ARCH = os.environ.get("AXP_OFFLOAD_ARCH", "gfx950")

COMMON = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-Wall", "-Wno-unused-function", "-Wno-unused-parameter", "-Wno-unused-variable"]


def _compile(src: str, obj: str) -> None:
    cmd = ["hipcc", *COMMON, "-c", src, "-o", obj]
    if src.endswith(".cpp"):
        cmd = ["hipcc", *COMMON, "-x", "hip", "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    warn = "\n".join(l for l in r.stderr.splitlines() if "packed-fp32-ops" not in l and l.strip())
    if warn.strip():
        sys.stderr.write(warn + "\n")


def _hip_runtime_link_args():
    """Link against the HIP runtime PyTorch loads (one runtime per process)."""
    try:
        import importlib.util
        spec = importlib.util.find_spec("torch")
        if spec is not None and spec.origin:
            tlib = os.path.join(os.path.dirname(spec.origin), "lib")
            if os.path.exists(os.path.join(tlib, "libamdhip64.so")):
                return [f"-L{tlib}", f"-Wl,-rpath,{tlib}", "-lamdhip64"]
    except Exception:
        pass
    return ["-L/opt/rocm/lib", "-Wl,-rpath,/opt/rocm/lib", "-lamdhip64"]


def build(verbose: bool = True) -> str:
    os.makedirs(OUT_DIR, exist_ok=True)
    obj_dir = os.path.join(OUT_DIR, "obj")
    os.makedirs(obj_dir, exist_ok=True)
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.cpp")) + glob.glob(os.path.join(CSRC, "*.hip")))
    objs = [os.path.join(obj_dir, os.path.basename(s) + ".o") for s in srcs]
    with cf.ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        list(ex.map(lambda a: _compile(*a), zip(srcs, objs)))
    tmp = LIB + f".tmp{os.getpid()}"
    # plain C++ link: the objects carry their gfx950 code; the HIP runtime comes from
    # the same library PyTorch uses so that streams and allocations are shared
    cmd = ["g++", "-shared", "-fPIC", "-o", tmp, *objs, *_hip_runtime_link_args(), "-lpthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}")
    return LIB


if __name__ == "__main__":
    build()
