"""Build libcpc.so for gfx950 in-tree.

    python -m paper_1205_6113_amd.build

HIP sources are compiled with hipcc for gfx950 with packed FP32 instructions
disabled; the Galerkin product (rap.hip) and the host setup are compiled without
FMA contraction (their results must be reproducible bit for bit).
"""
from __future__ import annotations

import os
import subprocess
import sys
from pathlib import Path

PKG = Path(__file__).resolve().parent
CSRC = PKG / "csrc"
INCLUDE = PKG.parent / "include"
BUILD = PKG / "_build"
LIB = PKG / "libcpc.so"
HOST_LIB = PKG / "libcpc_host.so"  # host-only SETUP code for CPU tests

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
DEVICE_FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
                "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                f"-I{INCLUDE}", "-Wno-unused-result"]

SOURCES = [
    # (source, compiler, extra flags)
    ("kernels.hip", "hip", []),
    ("sweep.hip", "hip", []),
    ("wave_sweep.hip", "hip", []),
    ("batch.hip", "hip", []),
    ("rap.hip", "hip", ["-ffp-contract=off"]),
    ("tpfa.hip", "hip", ["-ffp-contract=off"]),
    ("dense_tri.hip", "hip", []),
    ("dense_gemm.hip", "hip", []),
    ("noalloc.hip", "hip", []),
    ("host_setup.cpp", "gxx", ["-ffp-contract=off"]),
    ("solver.cpp", "hiphost", []),
]


def _cmd(src: Path, obj: Path, kind: str, extra):
    if kind == "hip":
        return [HIPCC, *DEVICE_FLAGS, *extra, "-c", str(src), "-o", str(obj)]
    if kind == "hiphost":
        return [HIPCC, "-O2", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", f"-I{INCLUDE}", *extra,
                "-c", str(src), "-o", str(obj)]
    return ["g++", "-O2", "-std=c++17", "-fPIC", f"-I{INCLUDE}", *extra, "-c", str(src), "-o", str(obj)]


def build(verbose: bool = False) -> Path:
    """Compile every source (always) and link libcpc.so."""
    BUILD.mkdir(exist_ok=True)
    procs = []
    objs = []
    for name, kind, extra in SOURCES:
        src = CSRC / name
        obj = BUILD / (name + ".o")
        objs.append(obj)
        cmd = _cmd(src, obj, kind, extra)
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((name, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
    failed = []
    for name, p in procs:
        out, _ = p.communicate()
        text = out.decode(errors="replace")
        lines = [ln for ln in text.splitlines() if "packed-fp32-ops" not in ln and ln.strip()]
        if p.returncode != 0:
            failed.append((name, "\n".join(lines)))
        elif verbose and lines:
            print("\n".join(lines))
    if failed:
        msg = "\n".join(f"--- {n}\n{t}" for n, t in failed)
        raise RuntimeError(f"build failed:\n{msg}")
    tmp = LIB.with_suffix(".so.tmp")
    cmd = [HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", str(tmp), *map(str, objs)]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    # host-only library of the SETUP code (no GPU needed), used by CPU tests
    tmp = HOST_LIB.with_suffix(".so.tmp")
    cmd = ["g++", "-O2", "-std=c++17", "-fPIC", "-shared", "-pthread", "-ffp-contract=off", f"-I{INCLUDE}", "-o", str(tmp),
           str(CSRC / "host_setup.cpp"), str(CSRC / "host_check.cpp")]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, HOST_LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
    print(LIB)
