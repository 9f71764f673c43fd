"""Builds the HIP library in-tree: csrc/*.hip -> paper_1308_4011_amd/libmm355.so (gfx950).

Usage: python -m paper_1308_4011_amd.build [--jobs N]
"""
from __future__ import annotations

import argparse
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libmm355.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

FLAGS = [
    "-O3", f"--offload-arch={ARCH}", "-fPIC", "-std=c++17",
    # no packed fp32 instructions anywhere in the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"), "-I", CSRC,
]

_NOISE = "is not a recognized feature for this target"


def _run(cmd):
    p = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    out = "\n".join(l for l in p.stdout.splitlines() if _NOISE not in l)
    return p.returncode, out


def build(jobs: int = 8, verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    srcs = sorted(f for f in os.listdir(CSRC) if f.endswith(".hip"))
    objs, procs = [], []
    for f in srcs:
        obj = os.path.join(BUILD, f[:-4] + ".o")
        objs.append(obj)
        cmd = [HIPCC, *FLAGS, "-c", os.path.join(CSRC, f), "-o", obj]
        procs.append((f, cmd))
    # compile in parallel
    running = []
    errors = []
    for f, cmd in procs:
        running.append((f, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)))
        if len(running) >= jobs:
            f0, p0 = running.pop(0)
            out = p0.communicate()[0]
            if p0.returncode:
                errors.append((f0, out))
            elif verbose and out.strip():
                print(out)
    for f0, p0 in running:
        out = p0.communicate()[0]
        if p0.returncode:
            errors.append((f0, out))
    if errors:
        msg = "\n".join(f"--- {f}\n" + "\n".join(l for l in o.splitlines() if _NOISE not in l) for f, o in errors)
        raise RuntimeError("HIP compile failed:\n" + msg)
    tmp = LIB + ".tmp"
    rc, out = _run([HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", *objs, "-o", tmp])
    if rc:
        raise RuntimeError("link failed:\n" + out)
    os.replace(tmp, LIB)
    return LIB


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=8)
    ap.add_argument("-v", action="store_true")
    a = ap.parse_args(argv)
    print(build(a.jobs, a.v))


if __name__ == "__main__":
    sys.exit(main())
