"""Build libhmc.so (HIP, gfx950) in-tree.

    python -m paper_1306_1821_amd.build

Each source is compiled to an object in its own hipcc process (in parallel),
then the objects are linked into the shared library.  Packed FP32 instructions
are disabled on purpose (-packed-fp32-ops); the library is plain hipcc output
for gfx950 only.
"""
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libhmc.so")
OBJDIR = os.path.join(HERE, "_build")
SOURCES = [os.path.join(HERE, "csrc", f) for f in ("kernels.hip", "runtime.hip", "cnn.hip")]
HIPCC = os.environ.get("HIPCC", shutil.which("hipcc") or "/opt/rocm/bin/hipcc")
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wno-unused-result", "-I", os.path.join(ROOT, "include")]


def build(verbose=True, out=LIB, defines=()):
    os.makedirs(OBJDIR, exist_ok=True)
    tag = os.path.splitext(os.path.basename(out))[0]
    procs = []
    objs = []
    for src in SOURCES:
        obj = os.path.join(OBJDIR, f"{tag}.{os.path.splitext(os.path.basename(src))[0]}.o")
        cmd = [HIPCC, *FLAGS, *[f"-D{d}" for d in defines], "-c", src, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((subprocess.Popen(cmd), cmd))
        objs.append(obj)
    for p, cmd in procs:
        if p.wait() != 0:
            raise subprocess.CalledProcessError(p.returncode, cmd)
    tmp = out + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    build()
    sys.exit(0)
