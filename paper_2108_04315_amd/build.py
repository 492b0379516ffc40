"""Builds libmisr.so (HIP, gfx950) in the package directory.

    python -m paper_2108_04315_amd.build [-v] [--incremental] [--sanitize]

The image kernels are compiled once per scale factor (-DMISR_SCALE=s); the
translation units compile in parallel.
"""
from __future__ import annotations

import hashlib
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libmisr.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950",
    # keep packed-FP32 instructions out of the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument", "-I", os.path.join(ROOT, "include"),
]


def _units():
    units = [("image_kernels.hip", [f"-DMISR_SCALE={s}"], f"_image_s{s}.o") for s in (1, 2, 3, 4)]
    units.append(("scalar_kernels.hip", [], "_scalar.o"))
    units.append(("general_kernels.hip", [], "_general.o"))
    units.append(("noalloc.hip", [], "_noalloc.o"))
    for src in ("abi.cpp", "server.cpp"):
        if os.path.exists(os.path.join(CSRC, src)):
            units.append((src, ["-x", "hip"], "_" + src.replace(".cpp", ".o")))
    return units


OBJ_CACHE = os.path.join(ROOT, "_build")


def _unit_hash(src: str, extra) -> str:
    """Hash of one unit's inputs: its source, every header it may include and
    the command line."""
    h = hashlib.sha256(" ".join([HIPCC] + FLAGS + list(extra)).encode())
    h.update(open(os.path.join(CSRC, src), "rb").read())
    for d in (CSRC, os.path.join(ROOT, "include")):
        for f in sorted(os.listdir(d)):
            if f.endswith(".h"):
                h.update(f.encode())
                h.update(open(os.path.join(d, f), "rb").read())
    return h.hexdigest()[:20]


# host code only: the device code is never built with a sanitizer
SAN_FLAGS = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-Xarch_host", "-fno-omit-frame-pointer", "-g"]


def build(verbose: bool = False, jobs: int | None = None, incremental: bool = False,
          sanitize: bool = False) -> str:
    """Compiles every unit and links libmisr.so.  incremental: reuse object
    files under _build/ whose unit hash is unchanged.  sanitize: link
    libmisr_san.so instead, its host code instrumented with AddressSanitizer
    and UndefinedBehaviorSanitizer (loaded when MISR_SANITIZE=1)."""
    jobs = jobs or min(8, os.cpu_count() or 4)
    os.makedirs(OBJ_CACHE, exist_ok=True)
    san = SAN_FLAGS if sanitize else []

    def compile_one(u):
        src, extra, obj = u
        extra = list(extra) + san
        out = os.path.join(OBJ_CACHE, f"{obj[:-2]}_{_unit_hash(src, extra)}.o")
        if incremental and os.path.exists(out):
            return out
        cmd = [HIPCC] + FLAGS + extra + ["-c", os.path.join(CSRC, src), "-o", out + ".tmp"]
        if verbose:
            print(" ".join(cmd), flush=True)
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"compile failed: {src} {extra}\n{r.stderr}")
        os.replace(out + ".tmp", out)
        return out

    units = _units()
    with ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(compile_one, units))
    lib = os.path.join(HERE, "libmisr_san.so") if sanitize else LIB
    tmp = lib + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs + ["-lpthread"]
    if sanitize:
        cmd += ["-Xarch_host", "-fsanitize=address,undefined", "-shared-libsan"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, lib)
    if sanitize:
        return lib
    keep = set(objs)
    for f in os.listdir(OBJ_CACHE):
        p = os.path.join(OBJ_CACHE, f)
        if p not in keep and f.endswith(".o"):
            os.remove(p)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv, incremental="--incremental" in sys.argv,
                sanitize="--sanitize" in sys.argv))
