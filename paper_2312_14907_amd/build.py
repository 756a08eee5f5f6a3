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
           "mpbp_frames_64.hip", "mpbp_frames_32.hip", "mpbp_frames_150.hip", "mpbp_device.hip", "mpbp_map.hip", "mpbp_plain.hip", "mpbp_unwrap.hip", "mpbp_host.cpp"]
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


def build(verbose=False, jobs=None, out=None, objdir=None, host_flags=(), rebuild=None, defines=()):
    """Compile every source to an object in parallel, then link libmpbp.so.

    out / objdir: another library path and object folder; host_flags: extra flags of the
    host compilation (each behind -Xarch_host); defines: preprocessor symbols (host and
    device); rebuild: the sources to compile (the others' objects are taken from the
    default object folder, which must be built)."""
    jobs = jobs or max(1, min(8, os.cpu_count() or 1))
    objdir = objdir or os.path.join(PKG, "_build")
    os.makedirs(objdir, exist_ok=True)
    hflags = [x for f in host_flags for x in ("-Xarch_host", f)] + [f"-D{d}" for d in defines]
    procs = []
    objs = []
    for src in SOURCES:
        if rebuild is not None and src not in rebuild:
            objs.append(os.path.join(PKG, "_build", src + ".o"))
            continue
        obj = os.path.join(objdir, src + ".o")
        objs.append(obj)
        cmd = [hipcc(), *FLAGS, *hflags, "-I", os.path.join(ROOT, "include"), "-c",
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
    lib = out or LIB
    tmp = lib + ".tmp"
    cmd = [hipcc(), *FLAGS, *hflags, "-shared", "-o", tmp, *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}")
    os.replace(tmp, lib)
    return lib


def _wait(item):
    src, p = item
    out, _ = p.communicate()
    text = out.decode(errors="replace")
    if p.returncode != 0:
        raise RuntimeError(f"compile of {src} failed:\n{text}")
    warn = [ln for ln in text.splitlines() if "warning" in ln and "packed-fp32-ops" not in ln]
    if warn:
        sys.stderr.write("\n".join(warn) + "\n")


DEBUG_LIB = os.path.join(PKG, "libmpbp_debug.so")


def build_debug(verbose=False):
    """libmpbp_debug.so: the library with the device-side bounds checks of the projection
    and the back-projection (MPBP_DEBUG); every compute call then waits and reports a check
    that fired as MPBP_ERR_INTERNAL.  The kernels with checks live in mpbp_device.hip, the
    status word's reader in mpbp_host.cpp; the other objects are the release build's."""
    return build(verbose=verbose, out=DEBUG_LIB, objdir=os.path.join(PKG, "_build_debug"),
                 rebuild=("mpbp_device.hip", "mpbp_host.cpp"), defines=("MPBP_DEBUG",))


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
    print(build_debug(verbose="-v" in sys.argv))
