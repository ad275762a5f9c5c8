"""Compile the HIP sources into the in-tree shared library librbl.so (gfx950).

Each source is compiled in two passes that share one compilation-unit id (-cuid), so that
the host pass registers the same (externalised) names of static device variables that
the device pass defines:
  1. device pass: gfx950 code object bundle (fat binary), built without packed FP32
     instruction selection (FP32 work is issued as scalar VALU operations);
  2. host pass: the x86-64 object, embedding that fat binary.
The packed-FP32 switch therefore reaches the device compiler only.
"""
import hashlib
import os
import shutil
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "librbl.so")
SOURCES = ["kernels.hip", "likelihood.hip", "api.hip", "serve.hip", "mala.hip", "noalloc.hip", "fullband.hip", "refsearch.hip"]

COMMON = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-result", "-pthread"]
DEVICE_ONLY = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def hipcc():
    exe = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(exe):
        raise RuntimeError("hipcc not found")
    return exe


def _cuid(src):
    return hashlib.sha256(src.encode()).hexdigest()[:16]


def _run_all(cmds, verbose):
    procs = []
    for cmd in cmds:
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((subprocess.Popen(cmd), cmd))
    failed = [cmd for p, cmd in procs if p.wait() != 0]
    if failed:
        raise subprocess.CalledProcessError(1, failed[0])


def build(verbose=False):
    """Compile every source and link librbl.so; returns the library path."""
    bdir = os.path.join(HERE, "_build")
    os.makedirs(bdir, exist_ok=True)
    dev_cmds, host_cmds, objs = [], [], []
    for src in SOURCES:
        path = os.path.join(CSRC, src)
        stem = os.path.join(bdir, src.replace(".hip", ""))
        cuid = f"-cuid={_cuid(src)}"
        fatbin = stem + ".hipfb"
        obj = stem + ".o"
        dev_cmds.append([hipcc(), *COMMON, *DEVICE_ONLY, cuid, "--cuda-device-only", path, "-o", fatbin])
        host_cmds.append([hipcc(), *COMMON, cuid, "--cuda-host-only", "-Xclang", "-fcuda-include-gpubinary",
                          "-Xclang", fatbin, "-c", path, "-o", obj])
        objs.append(obj)
    _run_all(dev_cmds, verbose)
    _run_all(host_cmds, verbose)
    tmp = LIB + ".tmp"
    cmd = [hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", "-pthread", *objs, "-o", tmp]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
