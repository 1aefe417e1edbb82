"""Builds the HIP library libadr.so (gfx950) in-tree."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libadr.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

CLANG = os.environ.get("ADR_CLANG", "/opt/rocm/lib/llvm/bin/clang++")


def runtime_dir() -> str:
    """Directory of the HIP runtime library used at run time (torch's)."""
    import importlib.util
    spec = importlib.util.find_spec("torch")
    if spec is None or not spec.origin:
        return "/opt/rocm/lib"
    d = os.path.join(os.path.dirname(spec.origin), "lib")
    return d if os.path.exists(os.path.join(d, "libamdhip64.so")) else "/opt/rocm/lib"


SOURCES = ["adr_geometry.cpp", "adr_kernels.hip", "adr_krylov.hip", "adr_api.cpp", "adr_tri.hip", "adr_tri_noalloc.hip", "adrnn.hip", "adr_probe.hip"]
FLAGS = ["-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC",
         # packed FP32 instructions stay off (see the design notes)
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-command-line-argument"]


def build(verbose: bool = False) -> str:
    objs = []
    procs = []
    for s in SOURCES:
        src = os.path.join(CSRC, s)
        obj = os.path.join(CSRC, os.path.splitext(s)[0] + ".o")
        lang = ["-x", "hip"] if s.endswith(".hip") else []
        cmd = [HIPCC, *FLAGS, *lang, "-c", src, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT), s))
        objs.append(obj)
    for p, s in procs:
        out, _ = p.communicate()
        text = out.decode(errors="replace")
        # the host pass does not know the packed-fp32 feature: harmless
        lines = [ln for ln in text.splitlines() if "packed-fp32-ops" not in ln and ln.strip()]
        if p.returncode != 0:
            raise RuntimeError(f"hipcc failed on {s}:\n{text}")
        if verbose and lines:
            print("\n".join(lines))
    tmp = LIB + ".tmp"
    # Link against the HIP runtime that torch loads, so that one process holds a
    # single runtime (torch provides the device memory and streams).
    rt_dir = runtime_dir()
    cmd = [CLANG, "-shared", "-fPIC", *objs, "-o", tmp, f"-L{rt_dir}", "-l:libamdhip64.so",
           f"-Wl,-rpath,{rt_dir}", "-lpthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + r.stdout + r.stderr)
    os.replace(tmp, LIB)
    for o in objs:
        os.remove(o)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
