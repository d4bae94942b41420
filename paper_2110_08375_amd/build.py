"""Compile the HIP library (gfx950) and the host build of its arithmetic header.

The library is built in-tree: ``paper_2110_08375_amd/libmdls.so`` from the translation
units in ``csrc/`` (one per precision, compiled in parallel, then linked), and
``paper_2110_08375_amd/libmdhost.so`` from ``csrc/md_host_shim.cpp`` (host compiler).
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libmdls.so")
HOSTLIB = os.path.join(PKG, "libmdhost.so")

UNITS = ["mdls_capi.hip", "mdls_p1.hip", "mdls_p2.hip", "mdls_p4.hip", "mdls_p8.hip"]
HIPFLAGS = [
    "-O3", "--offload-arch=gfx950", "-std=c++17", "-fPIC",
    # every + and * rounded on its own: the error-free transforms depend on it
    "-ffp-contract=off",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def _hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found: the MI355X library cannot be built")


def build_library(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    hipcc = _hipcc()
    procs = []
    objs = []
    for u in UNITS:
        obj = os.path.join(BUILD, u.replace(".hip", ".o"))
        objs.append(obj)
        cmd = [hipcc, *HIPFLAGS, "-I", INCLUDE, "-I", CSRC, "-c", os.path.join(CSRC, u), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((u, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
    failed = []
    for u, p in procs:
        out, _ = p.communicate()
        if p.returncode != 0:
            failed.append((u, out.decode(errors="replace")))
    if failed:
        raise RuntimeError("HIP compile failed:\n" + "\n".join("%s:\n%s" % f for f in failed))
    tmp = LIB + ".tmp%d" % os.getpid()
    subprocess.run([hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs], check=True)
    os.replace(tmp, LIB)
    return LIB


def build_host_shim() -> str:
    tmp = HOSTLIB + ".tmp%d" % os.getpid()
    cxx = shutil.which("g++") or "g++"
    subprocess.run([cxx, "-O2", "-std=c++17", "-fPIC", "-shared", "-ffp-contract=off", "-fno-fast-math",
                    "-Wno-unknown-pragmas", "-I", CSRC, "-o", tmp,
                    os.path.join(CSRC, "md_host_shim.cpp")], check=True)
    os.replace(tmp, HOSTLIB)
    return HOSTLIB


def build_all(verbose: bool = False):
    build_host_shim()
    return build_library(verbose=verbose)


if __name__ == "__main__":
    print(build_all(verbose="-v" in sys.argv))
