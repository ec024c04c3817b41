"""Builds libsketch.so for gfx950 in-tree with hipcc (one shared library:
HIP kernels + the C ABI of include/sketch.h)."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libsketch.so")
SOURCES = ["k_stream.hip", "k_core.hip", "k_mfma.hip", "k_coop.hip", "k_window.hip", "k_tri.hip", "k_trix.hip", "k_cholx.hip", "k_cod.hip", "sk_api.cpp",
           "sk_window.cpp", "sk_cod.cpp", "sk_server.cpp"]
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wno-unused-result", "-fvisibility=hidden"]


def sources():
    return [os.path.join(CSRC, s) for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]


def build(verbose=False, jobs=8):
    """Compile every source to an object in parallel, then link."""
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    procs = []
    objs = []
    for src in sources():
        obj = os.path.join(objdir, os.path.basename(src) + ".o")
        objs.append(obj)
        cmd = ["hipcc", "-x", "hip"] + [f for f in FLAGS if f != "-shared"] + ["-c", src, "-o", obj,
                                                                             "-I", CSRC]
        if verbose:
            print(" ".join(cmd))
        procs.append((src, subprocess.Popen(cmd, stderr=subprocess.PIPE, stdout=subprocess.PIPE)))
    failed = []
    for src, p in procs:
        out, err = p.communicate()
        msg = err.decode(errors="replace")
        msg = "\n".join(l for l in msg.splitlines() if "packed-fp32-ops" not in l)
        if p.returncode != 0:
            failed.append((src, msg))
        elif verbose and msg.strip():
            print(msg)
    if failed:
        for src, msg in failed:
            sys.stderr.write(f"--- {src}\n{msg}\n")
        raise RuntimeError("hipcc failed")
    cmd = ["hipcc", "--offload-arch=gfx950", "-shared", "-fPIC", "-o", LIB + ".tmp"] + objs
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
