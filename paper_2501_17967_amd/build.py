"""Build libvolpot.so (the C-ABI library) in-tree with hipcc for gfx950.

    python -m paper_2501_17967_amd.build

Host C++ sources and the HIP kernels are compiled separately (objects in _build/) and linked
into paper_2501_17967_amd/libvolpot.so. Always recompiles.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libvolpot.so")
BUILD = os.path.join(ROOT, "_build")
ARCH = os.environ.get("VOLPOT_ARCH", "gfx950")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
COMMON = ["-O3", "-std=c++17", "-fPIC", "-I" + os.path.join(ROOT, "include"), "-Wall", "-Wno-unused-result"]
DEVICE = ["--offload-arch=" + ARCH, "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def build(verbose=False):
    os.makedirs(BUILD, exist_ok=True)
    jobs = []
    objs = []
    for src in ("plan.cpp", "tables.cpp", "api.cpp", "tune.cpp", "tree.cpp", "strip.cpp"):
        obj = os.path.join(BUILD, src + ".o")
        cmd = [HIPCC] + COMMON + ["-c", os.path.join(CSRC, src), "-o", obj]
        jobs.append(cmd)
        objs.append(obj)
    for src in ("kernels.hip", "layer.hip", "points.hip", "tree.hip", "strip.hip", "strip_factor.hip", "moments.hip", "peak.hip"):
        kobj = os.path.join(BUILD, src + ".o")
        jobs.append([HIPCC] + COMMON + DEVICE + ["-c", os.path.join(CSRC, src), "-o", kobj])
        objs.append(kobj)
    procs = [(cmd, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)) for cmd in jobs]
    failed = False
    for cmd, p in procs:
        out, _ = p.communicate()
        text = out.decode(errors="replace")
        text = "\n".join(l for l in text.splitlines() if "packed-fp32-ops" not in l)
        if p.returncode != 0:
            failed = True
            sys.stderr.write("FAILED: %s\n%s\n" % (" ".join(cmd), text))
        elif verbose and text.strip():
            sys.stderr.write(text + "\n")
    if failed:
        raise RuntimeError("libvolpot build failed")
    tmp = OUT + ".tmp%d" % os.getpid()
    link = [HIPCC, "-shared", "-fPIC", "--offload-arch=" + ARCH, "-o", tmp] + objs + [
        "-L/opt/rocm/lib", "-lrocprofiler-sdk-roctx", "-lpthread"]
    r = subprocess.run(link, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)
    if r.returncode != 0:
        raise RuntimeError("libvolpot link failed:\n" + r.stdout.decode(errors="replace"))
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose=True))
