"""Build libconvreal.so (gfx950) in-tree with hipcc.

Run as ``python paper_1409_4441_amd/build.py`` (a script: importing the package would load the
library it builds). Every call recompiles.
"""
from __future__ import annotations

import os
import shlex
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libconvreal.so")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

# Packed FP32 VALU instructions are kept out of every kernel.
HIP_FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Wall", "-Wno-unused-function", "-I", os.path.join(ROOT, "include")]

SOURCES = ["capi.cpp", "split.cpp", "window.hip", "tabulate.hip", "plain.hip", "mixed.hip", "ringfft.hip", "mlp.hip", "sht.hip"]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(shlex.quote(c) for c in cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    out = (res.stdout or "") + (res.stderr or "")
    # hipcc's host pass does not know the packed-fp32 feature and says so; that line is noise.
    lines = [ln for ln in out.splitlines() if "packed-fp32-ops" not in ln]
    if res.returncode != 0:
        raise RuntimeError("build failed:\n" + "\n".join(lines))
    if verbose and lines:
        print("\n".join(lines))


# Host-side sanitizers for a checking build (every flag applies to the host pass only; the device
# code is built as usual): AddressSanitizer and UndefinedBehaviorSanitizer, errors fatal.
SANITIZE_COMPILE = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                    "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer"]
SANITIZE_LINK = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined", "-shared-libsan"]


def build(verbose: bool = False, jobs: int = 8, sanitize: bool = False, out_dir: str | None = None) -> str:
    """Compile every source and link libconvreal.so (in the package, or in out_dir). sanitize: the
    host code with ASan + UBSan (-O1 -g), for checking runs that preload the sanitizer runtime."""
    objdir = os.path.join(out_dir or HERE, "_build_san" if sanitize else "_build")
    os.makedirs(objdir, exist_ok=True)
    flags = HIP_FLAGS + (["-O1", "-g"] + SANITIZE_COMPILE if sanitize else [])
    objs = []
    procs = []
    for src in SOURCES:
        obj = os.path.join(objdir, os.path.splitext(src)[0] + ".o")
        objs.append(obj)
        lang = ["-x", "hip"] if src.endswith(".hip") else []
        cmd = [HIPCC] + flags + lang + ["-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(shlex.quote(c) for c in cmd), flush=True)
        procs.append((cmd, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)))
        if len(procs) >= jobs:
            _drain(procs)
    _drain(procs)
    lib = os.path.join(out_dir, "libconvreal.so") if out_dir else LIB
    tmp = lib + ".tmp"
    _run([HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC"] + (SANITIZE_LINK if sanitize else []) +
         ["-o", tmp] + objs, verbose)
    os.replace(tmp, lib)
    return lib


def _drain(procs):
    errors = []
    for cmd, pr in procs:
        out, _ = pr.communicate()
        lines = [ln for ln in (out or "").splitlines() if "packed-fp32-ops" not in ln]
        if pr.returncode != 0:
            errors.append(" ".join(cmd) + "\n" + "\n".join(lines))
        elif lines:
            print("\n".join(lines), file=sys.stderr)
    procs.clear()
    if errors:
        raise RuntimeError("build failed:\n" + "\n\n".join(errors))


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
