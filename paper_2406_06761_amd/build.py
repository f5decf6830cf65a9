"""Build libwally.so (HIP kernels + host library) for gfx950 with hipcc, in-tree."""
from __future__ import annotations

import os
import subprocess
import sys
from pathlib import Path

HERE = Path(__file__).resolve().parent
ROOT = HERE.parent
SRC = HERE / "csrc"
LIB = HERE / "libwally.so"
SOURCES = [SRC / "kernels.hip", SRC / "host.cpp"]
HEADERS = [SRC / "arith.h", SRC / "ntt.h", SRC / "kernels.h", SRC / "items.h", SRC / "plan.h", ROOT / "include" / "wally.h", ROOT / "include" / "wally_diag.h"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "--offload-arch=" + ARCH,
    # packed fp32 instructions are disabled for every HIP translation unit
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I" + str(ROOT / "include"), "-I" + str(SRC),
    "-Wall", "-Wno-unused-result",
]


def build(verbose: bool = False, out: Path = LIB, extra=()) -> Path:
    """Compile every source (always: the caller asks for a fresh build)."""
    objs = []
    tmpdir = HERE / "_build" / ("default" if not extra else "_".join(x.strip("-").replace("=", "") for x in extra))
    tmpdir.mkdir(parents=True, exist_ok=True)
    for src in SOURCES:
        obj = tmpdir / (src.name + ".o")
        lang = ["-x", "hip"] if src.suffix == ".hip" else ["-x", "hip"]
        cmd = [HIPCC, *FLAGS, *extra, *lang, "-c", str(src), "-o", str(obj)]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        objs.append(obj)
    tmp = out.with_suffix(".so.tmp%d" % os.getpid())
    cmd = [HIPCC, "--offload-arch=" + ARCH, "-shared", "-fPIC", *map(str, objs), "-o", str(tmp)]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
    print(LIB)
