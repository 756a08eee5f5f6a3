"""Build libmpbp.so (the C-ABI library of include/mpbp.h) for gfx950 in-tree.

    python -m paper_2312_14907_amd.build
"""
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libmpbp.so")
SOURCES = ["mpbp_frames_256.hip", "mpbp_frames_192.hip", "mpbp_frames_128.hip", "mpbp_frames_96.hip",
           "mpbp_frames_64.hip", "mpbp_frames_32.hip", "mpbp_frames_150.hip", "mpbp_device.hip", "mpbp_plain.hip", "mpbp_unwrap.hip", "mpbp_host.cpp"]
ARCH = os.environ.get("MPBP_OFFLOAD_ARCH", "gfx950")

# Packed FP32 instructions are disabled for all device code.
FLAGS = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-fno-signed-zeros",
    "-Wno-unused-command-line-argument",
]


def hipcc():
    p = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(p):
        raise RuntimeError("hipcc not found")
    return p


def build(verbose=False, jobs=None):
    """Compile every source to an object in parallel, then link libmpbp.so."""
    jobs = jobs or max(1, min(8, os.cpu_count() or 1))
    objdir = os.path.join(PKG, "_build")
    os.makedirs(objdir, exist_ok=True)
    procs = []
    objs = []
    for src in SOURCES:
        obj = os.path.join(objdir, src + ".o")
        objs.append(obj)
        cmd = [hipcc(), *FLAGS, "-I", os.path.join(ROOT, "include"), "-c",
               os.path.join(CSRC, src), "-o", obj]
        if src.endswith(".cpp"):
            cmd[1:1] = ["-x", "hip"]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
        if len(procs) >= jobs:
            _wait(procs.pop(0))
    while procs:
        _wait(procs.pop(0))
    tmp = LIB + ".tmp"
    cmd = [hipcc(), *FLAGS, "-shared", "-o", tmp, *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}")
    os.replace(tmp, LIB)
    return LIB


def _wait(item):
    src, p = item
    out, _ = p.communicate()
    text = out.decode(errors="replace")
    if p.returncode != 0:
        raise RuntimeError(f"compile of {src} failed:\n{text}")
    warn = [ln for ln in text.splitlines() if "warning" in ln and "packed-fp32-ops" not in ln]
    if warn:
        sys.stderr.write("\n".join(warn) + "\n")


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
