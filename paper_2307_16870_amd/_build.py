"""Build the HIP library ``_lib/libeamps.so`` for gfx950 with hipcc.

Usage: ``python paper_2307_16870_amd/_build.py`` (or ``__graft_entry__.build()``);
run it by path, not as ``-m``, so the package (which loads the library) is
not imported first.
Every call recompiles all sources (one hipcc process per source, in
parallel) and links them into one shared library.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIBDIR = os.path.join(PKG, "_lib")
OBJDIR = os.path.join(PKG, "_build")
LIBNAME = "libeamps.so"

SOURCES = ["k_linalg.hip", "k_theta3.hip", "k_jacobi.hip", "k_jacobi2.hip", "k_observe.hip", "k_small.hip", "k_adjoint.hip",
           "k_qr.hip", "k_zgemm.hip", "k_chol.hip", "k_vidal.hip", "k_topk.hip", "ea_api.hip", "ea_adjoint.hip"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = os.environ.get("EA_OFFLOAD_ARCH", "gfx950")
FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-fPIC", "-std=c++17",
    # no packed FP32 instructions anywhere in the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
    f"-I{INCLUDE}", f"-I{CSRC}",
]


def _run(cmd):
    p = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    out = "\n".join(l for l in p.stdout.splitlines()
                    if "packed-fp32-ops" not in l and "not a recognized feature" not in l)
    return p.returncode, out


def build(verbose: bool = True) -> str:
    os.makedirs(LIBDIR, exist_ok=True)
    os.makedirs(OBJDIR, exist_ok=True)
    objs = []
    cmds = []
    for src in SOURCES:
        obj = os.path.join(OBJDIR, src.replace(".hip", ".o"))
        objs.append(obj)
        cmds.append([HIPCC, *FLAGS, "-c", os.path.join(CSRC, src), "-o", obj])
    with ThreadPoolExecutor(max_workers=min(8, len(cmds))) as ex:
        results = list(ex.map(_run, cmds))
    failed = False
    for cmd, (rc, out) in zip(cmds, results):
        if out.strip() and (verbose or rc):
            print(out, file=sys.stderr)
        if rc:
            failed = True
            print("FAILED:", " ".join(cmd), file=sys.stderr)
    if failed:
        raise RuntimeError("hipcc compilation failed")
    tmp = os.path.join(LIBDIR, LIBNAME + ".tmp")
    rc, out = _run([HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp])
    if rc:
        print(out, file=sys.stderr)
        raise RuntimeError("link failed")
    final = os.path.join(LIBDIR, LIBNAME)
    os.replace(tmp, final)
    shutil.rmtree(OBJDIR, ignore_errors=True)
    if verbose:
        print("built", final)
    return final


if __name__ == "__main__":
    build()
