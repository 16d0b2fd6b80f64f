"""Build the HIP solver library (libipoisson.so) for gfx950 with hipcc.

Run as ``python -m paper_2108_11871_amd.build``; ``__graft_entry__.build()``
calls :func:`build`.  The library is written next to this file.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
SOURCES = ["kernels.hip", "pass.hip", "conv.hip", "adjoint.hip", "screen.hip", "plan.hip"]
LIB = os.path.join(HERE, "libipoisson.so")
ARCH = os.environ.get("IPS_OFFLOAD_ARCH", "gfx950")


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def compile_flags():
    return [
        "-O3",
        "-std=c++17",
        "--offload-arch=" + ARCH,
        "-fPIC",
        # keep packed-FP32 instructions out of the generated code
        "-Xclang",
        "-target-feature",
        "-Xclang",
        "-packed-fp32-ops",
        "-I" + os.path.join(ROOT, "include"),
        "-I" + CSRC,
    ]


def build(verbose: bool = False) -> str:
    """Compile every HIP source and link libipoisson.so (always rebuilds)."""
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    objs = []
    procs = []
    for src in SOURCES:
        obj = os.path.join(objdir, src.replace(".hip", ".o"))
        cmd = [hipcc()] + compile_flags() + ["-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT), src))
        objs.append(obj)
    for proc, src in procs:
        out, _ = proc.communicate()
        if proc.returncode != 0:
            sys.stderr.write(out.decode(errors="replace"))
            raise RuntimeError("hipcc failed on %s" % src)
        elif verbose and out:
            sys.stderr.write(out.decode(errors="replace"))
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [hipcc(), "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp] + objs
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


def build_host_check(verbose: bool = False) -> str:
    """The sanitizer build of the host code: plan.hip compiled with
    AddressSanitizer and UndefinedBehaviorSanitizer on its host side only (the
    device code is built as usual), linked with the other objects of the
    library and the host-only driver tests/host_check.cpp into one program.
    Returns the program's path."""
    objdir = os.path.join(HERE, "_build")
    if not all(os.path.exists(os.path.join(objdir, s.replace(".hip", ".o"))) for s in SOURCES):
        build(verbose)
    sdir = os.path.join(objdir, "sanitize")
    os.makedirs(sdir, exist_ok=True)
    san = []
    for f in ("-fsanitize=address", "-fsanitize=undefined", "-fno-sanitize-recover=undefined",
              "-fno-omit-frame-pointer"):
        san += ["-Xarch_host", f]
    plan_o = os.path.join(sdir, "plan.o")
    cmd = [hipcc()] + compile_flags() + ["-g"] + san + ["-c", os.path.join(CSRC, "plan.hip"), "-o", plan_o]
    subprocess.check_call(cmd, stdout=subprocess.DEVNULL if not verbose else None,
                          stderr=subprocess.DEVNULL if not verbose else None)
    drv_o = os.path.join(sdir, "host_check.o")
    subprocess.check_call(["g++", "-std=c++17", "-g", "-fsanitize=address,undefined", "-fno-omit-frame-pointer",
                           "-I" + os.path.join(ROOT, "include"), "-c",
                           os.path.join(ROOT, "tests", "host_check.cpp"), "-o", drv_o])
    exe = os.path.join(sdir, "ips_host_check")
    objs = [os.path.join(objdir, s.replace(".hip", ".o")) for s in SOURCES if s != "plan.hip"]
    subprocess.check_call([hipcc(), "--offload-arch=" + ARCH] + san + ["-o", exe, drv_o, plan_o] + objs)
    return exe


if __name__ == "__main__":
    print(build(verbose=True))
